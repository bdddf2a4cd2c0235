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
//     parts in a K-blocked layout [row block of 32][column][32 rows].  Inside
//     a column the 32 values are placed so that the matrix-core fragments
//     can be read from LDS without bank conflicts: FP32 puts rows g, g+4, ...,
//     g+28 next to each other (one lane's eight k-steps) and XORs the 16-byte
//     slot index with column bits 1-3; bfloat16 parts XOR the slot of eight
//     consecutive rows with column bits 2-3.
//  2. MFMA: 128 x 128 lower-triangle tiles, split-K over row blocks, 4 waves x
//     (4 x 4 blocks of 16 x 16).  A row block of a 128-column panel is one
//     contiguous chunk (16 KB FP32, 8 KB per bfloat16 part) that goes from
//     HBM straight into LDS by LDS-DMA buffer loads, double buffered (the
//     loads of block b+1 fly while block b feeds the matrix cores); float32
//     accumulation over slabs of 512 rows, slabs added into float64
//     accumulators; split partials summed in float64 by the shared kernel.
//     BF16X6 runs the same stages on 256 x 128 tiles with 8 waves (two per
//     SIMD), which bring in half the panel bytes per product.
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
  int vec;                // Q and ldq allow 16-byte row loads
  float* pf;              // FP32 part
  unsigned short* p0;     // hi
  unsigned short* p1;     // lo (x3) / mid (x6)
  unsigned short* p2;     // lo (x6)
};

// The packed layout of a 32-row block in column cc.  FP32: the rows
// {g, g+4, ..., g+28} of k-step lane group g take positions 8g..8g+7, and
// the column's eight 16-byte slots are XORed with (cc >> 1) & 7 (row rr sits
// at position p = 8 (rr & 3) + (rr >> 2), slot (p >> 2) ^ ((cc >> 1) & 7)).
// bfloat16: rows 8s..8s+7 fill 16-byte slot s, XORed with (cc >> 2) & 3.
// Sixteen consecutive columns reading the same logical slot then hit sixteen
// different 16-byte bank groups.

// One workgroup packs a 32-row block x 128 columns: reads rows (coalesced,
// all 16 loads of a thread in flight together), transforms with the block's
// per-row mean and reciprocal scale (an LDS table), transposes through LDS,
// and writes whole 16-byte slots of the packed layout: FP32 gathers the four
// rows {g, g+4, g+8, g+12} (+16) of a slot, bfloat16 eight consecutive rows.
__global__ __launch_bounds__(256) void pack_kernel(PackArgs a) {
  __shared__ float tile[KB][BT + 1];
  __shared__ double rmu[KB], rinv[KB];
  const int64_t blk = blockIdx.x;
  const int64_t c0 = int64_t(blockIdx.y) * BT;
  const int tid = threadIdx.x;
  if (tid < KB) {
    const int64_t row = blk * KB + tid;
    const int64_t rowc = row < a.n ? row : a.n - 1;
    int vv = 0;
    while (vv + 1 < a.nvars && rowc >= a.row0[vv + 1]) ++vv;
    rmu[tid] = a.mean ? a.mean[rowc] : 0.0;
    rinv[tid] = a.scale ? 1.0 / a.scale[vv] : 1.0;
  }
  if (a.vec && c0 + BT <= a.k) {
    // whole tile in range, rows 16-byte aligned: thread -> 4 consecutive
    // columns 4 cq.. of rows rq + 8 i (four 16-byte loads, all in flight)
    const int cq = tid % (BT / 4), rq = tid / (BT / 4);
    flt4 q4[KB / 8];
#pragma unroll
    for (int i = 0; i < KB / 8; ++i) {
      const int64_t row = blk * KB + rq + 8 * i;
      q4[i] = *reinterpret_cast<const flt4*>(a.Q + (row < a.n ? row : a.n - 1) * a.ldq + c0 + 4 * cq);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KB / 8; ++i) {
      const int rr = rq + 8 * i;
      const bool rin = blk * KB + rr < a.n;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        tile[rr][4 * cq + e] =
            rin ? static_cast<float>((static_cast<double>(q4[i][e]) - rmu[rr]) * rinv[rr]) : 0.f;
    }
  } else {
    const int cc = tid % BT;
    const int64_t col = c0 + cc;
    const bool cin = col < a.k;
    const int64_t colc = cin ? col : 0;
    float q[KB / 2];
#pragma unroll
    for (int i = 0; i < KB / 2; ++i) {
      const int64_t row = blk * KB + tid / BT + 2 * i;
      q[i] = a.Q[(row < a.n ? row : a.n - 1) * a.ldq + colc];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KB / 2; ++i) {
      const int rr = tid / BT + 2 * i;
      const int64_t row = blk * KB + rr;
      float v = 0.f;
      if (row < a.n && cin) v = static_cast<float>((static_cast<double>(q[i]) - rmu[rr]) * rinv[rr]);
      tile[rr][cc] = v;
    }
  }
  __syncthreads();
  if (a.algo == 0) {
    // slot g of column c holds rows (g >> 1) + 4 j + 16 (g & 1), j = 0..3 (the FP32 layout above)
#pragma unroll
    for (int i = 0; i < BT * 8 / 256; ++i) {
      const int t = tid + 256 * i, cw = t >> 3, g = t & 7;
      flt4 x;
#pragma unroll
      for (int j = 0; j < 4; ++j) x[j] = tile[(g >> 1) + 4 * j + 16 * (g & 1)][cw];
      const size_t o = (size_t(blk) * a.kp + c0 + cw) * KB + ((g ^ ((cw >> 1) & 7)) << 2);
      *reinterpret_cast<flt4*>(a.pf + o) = x;
    }
  } else {
    // slot g of column c holds rows 8 g .. 8 g + 7 (the bfloat16 layout above)
#pragma unroll
    for (int i = 0; i < BT * 4 / 256; ++i) {
      const int t = tid + 256 * i, cw = t >> 2, g = t & 3;
      us8 h, m, l;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float x = tile[8 * g + j][cw];
        const unsigned short hh = bf16_rn_bits(x);
        const float r1 = x - bf16_to_f(hh);
        const unsigned short mm = bf16_rn_bits(r1);
        h[j] = hh;
        m[j] = mm;
        l[j] = bf16_rn_bits(r1 - bf16_to_f(mm));
      }
      const size_t o = (size_t(blk) * a.kp + c0 + cw) * KB + ((g ^ ((cw >> 2) & 3)) << 3);
      *reinterpret_cast<us8*>(a.p0 + o) = h;
      *reinterpret_cast<us8*>(a.p1 + o) = m;
      if (a.algo == 2) *reinterpret_cast<us8*>(a.p2 + o) = l;
    }
  }
}

struct MmaArgs {
  int64_t nb;     // row blocks
  int64_t kp;
  int ntiles, nsplit, xcd_map;
  int sel;        // tiles of the launch: 0 the whole lower triangle, 1 below the diagonal, 2 on it
  int nlaunch;    // tiles per split in the launch
  int64_t blocks_per_split;
  const float* pf;
  const unsigned short* p0;
  const unsigned short* p1;
  const unsigned short* p2;
  double* part;
};

// f32 16x16 MFMA output layout: lane l, element e -> row 4 (l / 16) + e, column l % 16
__device__ __forceinline__ int out_row(int lane, int e) { return 4 * (lane >> 4) + e; }

#define DOPINF_LDS(p) ((__attribute__((address_space(3))) void*)(p))

__device__ __forceinline__ __amdgpu_buffer_rsrc_t span_rsrc(const void* p, int nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, nbytes, 0x00020000);
}

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

template <int ALGO>
struct PackedGeom {
  static constexpr int NPART = ALGO == 0 ? 1 : (ALGO == 1 ? 2 : 3);
  static constexpr int ELT = ALGO == 0 ? 4 : 2;
  static constexpr int COLB = KB * ELT;             // bytes of one column of a block
  static constexpr int PANEL = BT * COLB;           // bytes of one panel part of a block
  static constexpr int CHUNKS = PANEL / 1024;       // 1 KB LDS-DMA chunks per panel part
  static constexpr int STAGE = 2 * NPART * PANEL;   // A and B panels, all parts
  static constexpr int NSTAGE = 2;                  // LDS stages (loads of one in flight)
  static_assert(CHUNKS % 4 == 0, "chunks per wave");
};

// Blocks of 16 x 16 that wave w (0..3) computes in a diagonal tile of the
// FP32 form: block columns w (block rows w..7) and 7 - w (block rows
// 7 - w..7), 9 blocks that cover the tile's 36 lower blocks over the four
// waves; block p sits in accumulator p (acc[p / 4][p % 4]).
__device__ __forceinline__ void diag_block(int w, int p, int& br, int& bc) {
  const bool first = p < 8 - w;
  br = first ? w + p : p - 1;
  bc = first ? w : 7 - w;
}

// One FP32 stage of wave W of a diagonal tile: the fragments of block rows
// W..7 are read once and serve as A and as the two B columns (rows W and
// 7 - W).  SA: the stage's panel, (o0, o1): the lane's two 16-byte slots.
template <int W, int COLB>
__device__ __forceinline__ void diag_stage_f32(const unsigned char* SA, int cm, int o0, int o1, flt4 (&acc)[4][4]) {
  flt4 f[8 - W][2];
#pragma unroll
  for (int i = 0; i < 8 - W; ++i) {
    const unsigned char* colp = SA + ((W + i) * 16 + cm) * COLB;
    f[i][0] = *reinterpret_cast<const flt4*>(colp + o0);
    f[i][1] = *reinterpret_cast<const flt4*>(colp + o1);
  }
#pragma unroll
  for (int kk = 0; kk < KB / 4; ++kk) {
#pragma unroll
    for (int p = 0; p < 8 - W; ++p)  // (W + p, W)
      acc[p >> 2][p & 3] =
          __builtin_amdgcn_mfma_f32_16x16x4f32(f[p][kk >> 2][kk & 3], f[0][kk >> 2][kk & 3], acc[p >> 2][p & 3], 0, 0, 0);
#pragma unroll
    for (int q = 0; q <= W; ++q) {  // (7 - W + q, 7 - W), p = 8 - W + q
      const int p = 8 - W + q;
      acc[p >> 2][p & 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(f[7 - 2 * W + q][kk >> 2][kk & 3],
                                                                f[7 - 2 * W][kk >> 2][kk & 3], acc[p >> 2][p & 3], 0, 0, 0);
    }
  }
}

template <int ALGO, bool DIAG, bool D9 = false>
__device__ __forceinline__ void packed_tile(const MmaArgs& g, int64_t b_lo, int64_t nst, int64_t a0, int64_t c0,
                                            unsigned char* smem, flt4 (&acc)[4][4], double (&acc64)[4][4][4]) {
  using Gm = PackedGeom<ALGO>;
  constexpr int NPART = Gm::NPART;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int wm = w >> 1, wn = w & 1;
  const uint32_t voff = uint32_t(lane) * 16;

  // chunk q of panel part (part, side) of block blk -> LDS slot
  auto issue = [&](int64_t st) {
    unsigned char* S = smem + (st % Gm::NSTAGE) * Gm::STAGE;
    const int64_t blk = b_lo + st;
#pragma unroll
    for (int part = 0; part < NPART; ++part) {
      const unsigned char* P = reinterpret_cast<const unsigned char*>(
          ALGO == 0 ? static_cast<const void*>(g.pf)
                    : static_cast<const void*>(part == 0 ? g.p0 : (part == 1 ? g.p1 : g.p2)));
      const unsigned char* rowblk = P + size_t(blk) * size_t(g.kp) * Gm::COLB;
#pragma unroll
      for (int side = 0; side < (DIAG ? 1 : 2); ++side) {
        const int64_t col0 = side == 0 ? a0 : c0;
        const unsigned char* src = rowblk + size_t(col0) * Gm::COLB;
        unsigned char* dst = S + (side * NPART + part) * Gm::PANEL;
        // the wave's share of the panel's chunks
#pragma unroll
        for (int t = 0; t < Gm::CHUNKS / 4; ++t) {
          const int q = w + 4 * t;
          const __amdgpu_buffer_rsrc_t rs = span_rsrc(src + q * 1024, 1024);
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, DOPINF_LDS(dst + q * 1024), 16, voff, 0, 0, 0);
        }
      }
    }
  };

  const int cm = lane & 15;
  const int gq = lane >> 4;
  constexpr int NS = Gm::NSTAGE;
  // LDS-DMA instructions one wave issues per stage
  constexpr int PER = NPART * (DIAG ? 1 : 2) * (Gm::CHUNKS / 4);
  for (int64_t p = 0; p < NS - 1 && p < nst; ++p) issue(p);
  // slabs of SLAB_STAGES stages: the inner loop has no branch on the
  // accumulators, so they stay in the registers the MFMAs write
  for (int64_t s0 = 0; s0 < nst; s0 += SLAB_STAGES) {
  const int64_t s1 = s0 + SLAB_STAGES < nst ? s0 + SLAB_STAGES : nst;
  for (int64_t st = s0; st < s1; ++st) {
    // stage st has landed once at most the later stages' loads are outstanding
    // (loads to LDS complete in issue order)
    if (NS > 2 && st + 1 < nst)
      wait_vmem<PER>();
    else
      wait_vmem<0>();
    barrier_only();
    // the buffer of stage st + NS - 1 was read in iteration st - 1, which every
    // wave has left at the barrier above
    if (st + NS - 1 < nst) issue(st + NS - 1);
    const unsigned char* S = smem + (st % NS) * Gm::STAGE;
    const unsigned char* SA = S;
    const unsigned char* SB = DIAG ? S : S + NPART * Gm::PANEL;
    if constexpr (ALGO == 0 && D9) {
      const int h = (cm >> 1) & 7;
      const int o0 = 16 * ((2 * gq) ^ h), o1 = 16 * ((2 * gq + 1) ^ h);
      switch (w) {  // w is wave-uniform: each wave runs the schedule of its own w
        case 0: diag_stage_f32<0, Gm::COLB>(SA, cm, o0, o1, acc); break;
        case 1: diag_stage_f32<1, Gm::COLB>(SA, cm, o0, o1, acc); break;
        case 2: diag_stage_f32<2, Gm::COLB>(SA, cm, o0, o1, acc); break;
        default: diag_stage_f32<3, Gm::COLB>(SA, cm, o0, o1, acc); break;
      }
    } else if constexpr (ALGO == 0) {
      // lane group gq holds rows gq, gq+4, ..., gq+28 of its column in slots 2gq, 2gq+1
      const int h = (cm >> 1) & 7;
      const int o0 = 16 * ((2 * gq) ^ h), o1 = 16 * ((2 * gq + 1) ^ h);
      flt4 af[4][2], bf[4][2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const unsigned char* colp = SA + (wm * 64 + i * 16 + cm) * Gm::COLB;
        af[i][0] = *reinterpret_cast<const flt4*>(colp + o0);
        af[i][1] = *reinterpret_cast<const flt4*>(colp + o1);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const unsigned char* colp = SB + (wn * 64 + j * 16 + cm) * Gm::COLB;
        bf[j][0] = *reinterpret_cast<const flt4*>(colp + o0);
        bf[j][1] = *reinterpret_cast<const flt4*>(colp + o1);
      }
#pragma unroll
      for (int kk = 0; kk < KB / 4; ++kk)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][kk >> 2][kk & 3], bf[j][kk >> 2][kk & 3],
                                                            acc[i][j], 0, 0, 0);
    } else {
      const int o = 16 * (gq ^ ((cm >> 2) & 3));
      bf16x8 a[NPART][4], b[NPART][4];
#pragma unroll
      for (int q = 0; q < NPART; ++q) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          a[q][i] = __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const us8*>(SA + q * Gm::PANEL + (wm * 64 + i * 16 + cm) * Gm::COLB + o));
#pragma unroll
        for (int j = 0; j < 4; ++j)
          b[q][j] = __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const us8*>(SB + q * Gm::PANEL + (wn * 64 + j * 16 + cm) * Gm::COLB + o));
      }
      // BF16X3's products lo.hi, hi.lo, hi.hi in the outer loop (smallest
      // first): 16 independent blocks lie between two products into one
      // accumulator, so no MFMA waits on the result of the previous one
      // (BF16X6 runs on gram_wide_kernel)
      constexpr int PA[3] = {1, 0, 0}, PB[3] = {0, 1, 0};
#pragma unroll
      for (int pr = 0; pr < 3; ++pr)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[PA[pr]][i], b[PB[pr]][j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int e = 0; e < 4; ++e) acc64[i][j][e] += static_cast<double>(acc[i][j][e]);
      acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
    }
  }
}

// sel 0: every lower-triangle tile, diagonal ones in the quadrant layout.
// The FP32 form splits the triangle like the FP64 Gram: the tiles below the
// diagonal (sel 1) fill whole rounds of resident workgroups, and the
// diagonal tiles (sel 2, D9) take a launch of their own in which each wave
// computes only 9 of the 36 lower 16 x 16 blocks.
template <int ALGO, bool D9 = false>
__global__ __launch_bounds__(NTH, 2) void gram_packed_kernel(MmaArgs g) {
  static_assert(ALGO < 2, "BF16X6 runs on gram_wide_kernel");
  __shared__ __attribute__((aligned(16))) unsigned char smem[PackedGeom<ALGO>::NSTAGE * PackedGeom<ALGO>::STAGE];
  int t, s;
  {
    const int bid = blockIdx.x;
    int tl;
    if (g.xcd_map) {
      const int xcd = bid & 7;
      const int local = bid >> 3;
      s = (local / g.nlaunch) * 8 + xcd;
      tl = local % g.nlaunch;
    } else {
      s = bid / g.nlaunch;
      tl = bid % g.nlaunch;
    }
    t = tl;
    if (g.sel == 1) {  // tl-th tile strictly below the diagonal
      int i, j;
      gramplan::tri_coords(tl, i, j);
      t = (i + 1) * (i + 2) / 2 + j;
    } else if (g.sel == 2) {
      t = tl * (tl + 1) / 2 + tl;
    }
  }
  int I, J;
  gramplan::tri_coords(t, I, J);
  const int64_t b_lo = int64_t(s) * g.blocks_per_split;
  const int64_t b_hi = min(g.nb, b_lo + g.blocks_per_split);
  const int64_t nst = b_hi > b_lo ? b_hi - b_lo : 0;
  const int64_t a0 = int64_t(I) * BT, c0 = int64_t(J) * BT;

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
  if (D9)
    packed_tile<ALGO, true, true>(g, b_lo, nst, a0, c0, smem, acc, acc64);
  else if (I == J)
    packed_tile<ALGO, true>(g, b_lo, nst, a0, c0, smem, acc, acc64);
  else
    packed_tile<ALGO, false>(g, b_lo, nst, a0, c0, smem, acc, acc64);

  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1;
  double* out = g.part + (size_t(s) * g.ntiles + t) * (BT * BT);
  if (D9) {  // the diagonal tile's lower blocks only (the reduction reads nothing above)
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      int br, bc;
      diag_block(w, p, br, bc);
#pragma unroll
      for (int e = 0; e < 4; ++e)
        out[(br * 16 + out_row(lane, e)) * BT + bc * 16 + (lane & 15)] = acc64[p >> 2][p & 3][e];
    }
    return;
  }
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

// The BF16X6 form on 256 x 128 tiles: a workgroup of 8 waves (two per
// SIMD) computes rows [256 I, 256 I + 256) (panel A) by columns
// [128 J, 128 J + 128) (panel B), J <= 2 I + 1, i.e. the 128 x 128 tiles
// (2 I, J) and (2 I + 1, J) of the lower triangle; tile t lies in row
// I = floor((sqrt(4 t + 1) - 1) / 2), J = t - I (I + 1).  Wave w computes rows
// 64 (w / 2) .. + 63 and columns 64 (w % 2) .. + 63 of the tile, skipping the
// stage's work when its quadrant lies above the diagonal or past k.  Against
// 128 x 128 tiles a row block's panels feed twice the products per byte
// brought in, and two waves per SIMD hide each other's LDS reads.
constexpr int WMT = 512;

template <int ALGO>
struct WideGeom {
  static constexpr int NPART = ALGO == 1 ? 2 : 3;
  static constexpr int COLB = KB * 2;            // bytes of one column of a block (one part)
  static constexpr int PA = 2 * BT * COLB;       // panel A part of a block (256 columns)
  static constexpr int PB = BT * COLB;           // panel B part of a block (128 columns)
  static constexpr int STAGE = NPART * (PA + PB);
  static constexpr int CHUNKS = STAGE / 1024;    // 1 KB LDS-DMA chunks per stage
  static_assert(CHUNKS % (WMT / 64) == 0, "chunks per wave");
};

struct WideArgs {
  int64_t nb, kp;
  int T, nwide, nsplit, xcd_map;
  int64_t bps;
  const unsigned short* part_p[3];  // hi, mid/lo, lo
  double* part;                     // per split, the T (T + 1) / 2 lower 128 x 128 tiles
};

template <int ALGO>
__global__ __launch_bounds__(WMT, 1) void gram_wide_kernel(WideArgs g) {
  using Gm = WideGeom<ALGO>;
  constexpr int NPART = Gm::NPART;
  __shared__ __attribute__((aligned(16))) unsigned char smem[2 * Gm::STAGE];
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
  const int64_t a0 = int64_t(I) * 2 * BT, c0 = int64_t(J) * BT;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int wm = w >> 1, wn = w & 1;
  const int sub = 2 * I + (wm >> 1);
  const bool live = sub < g.T && J <= sub;
  const uint32_t voff = uint32_t(lane) * 16;
  // stage layout: A parts (16 chunks each), then B parts (8 chunks each);
  // wave w issues chunks w, w + 8, ...
  auto issue = [&](int64_t st) {
    unsigned char* S = smem + (st & 1) * Gm::STAGE;
    const size_t blk = size_t(b_lo + st);
#pragma unroll
    for (int t = 0; t < Gm::CHUNKS / (WMT / 64); ++t) {
      const int q = w + (WMT / 64) * t;
      const bool isa = q < NPART * (Gm::PA / 1024);
      const int qa = isa ? q : q - NPART * (Gm::PA / 1024);
      const int pt = isa ? qa / (Gm::PA / 1024) : qa / (Gm::PB / 1024);
      const int qc = isa ? qa % (Gm::PA / 1024) : qa % (Gm::PB / 1024);
      const unsigned char* src = reinterpret_cast<const unsigned char*>(g.part_p[pt]) +
                                 (blk * size_t(g.kp) + size_t(isa ? a0 : c0)) * Gm::COLB + qc * 1024;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(span_rsrc(src, 1024), DOPINF_LDS(S + q * 1024), 16, voff, 0, 0, 0);
    }
  };
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
  const int cm = lane & 15, gq = lane >> 4;
  const int o = 16 * (gq ^ ((cm >> 2) & 3));
  if (nst > 0) issue(0);
  // slabs of SLAB_STAGES stages: float32 sums over at most 512 rows, then the
  // float64 accumulators
  for (int64_t s0 = 0; s0 < nst; s0 += SLAB_STAGES) {
    const int64_t s1 = s0 + SLAB_STAGES < nst ? s0 + SLAB_STAGES : nst;
    for (int64_t st = s0; st < s1; ++st) {
      wait_vmem<0>();
      barrier_only();
      // the other buffer was read in iteration st - 1, which every wave has left
      if (st + 1 < nst) issue(st + 1);
      if (!live) continue;  // wave-uniform
      const unsigned char* SA = smem + (st & 1) * Gm::STAGE;
      const unsigned char* SB = SA + NPART * Gm::PA;
      bf16x8 a[NPART][4], b[NPART][4];
#pragma unroll
      for (int q = 0; q < NPART; ++q) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          a[q][i] = __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const us8*>(SA + q * Gm::PA + (wm * 64 + i * 16 + cm) * Gm::COLB + o));
#pragma unroll
        for (int j = 0; j < 4; ++j)
          b[q][j] = __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const us8*>(SB + q * Gm::PB + (wn * 64 + j * 16 + cm) * Gm::COLB + o));
      }
      // products in the outer loop (smallest first), as in packed_tile
      constexpr int PA_[6] = {2, 0, 1, 1, 0, 0}, PB_[6] = {0, 2, 1, 0, 1, 0};
#pragma unroll
      for (int pr = (ALGO == 2 ? 0 : 3); pr < 6; ++pr)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[PA_[pr]][i], b[PB_[pr]][j], acc[i][j], 0, 0, 0);
    }
    if (live) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
          for (int e = 0; e < 4; ++e) acc64[i][j][e] += static_cast<double>(acc[i][j][e]);
          acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
        }
    }
  }
  if (!live) return;
  const int ntiles = g.T * (g.T + 1) / 2;
  double* out = g.part + (size_t(s) * ntiles + size_t(sub) * (sub + 1) / 2 + J) * (BT * BT);
  const int r0 = (wm & 1) * 64;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        out[(r0 + i * 16 + out_row(lane, e)) * BT + wn * 64 + j * 16 + (lane & 15)] = acc64[i][j][e];
}

int tiles_of(int64_t m) { return int((m + BT - 1) / BT); }
int nparts(int algo) { return algo == DOPINF_GRAM_NATIVE ? 1 : (algo == DOPINF_GRAM_BF16X3 ? 2 : 3); }
size_t part_elt(int algo) { return algo == DOPINF_GRAM_NATIVE ? 4 : 2; }

struct LowpPlan {
  int64_t nb, kp;
  int T, ntiles, nwide, nsplit;
  int64_t bps;
  size_t pack_bytes, part_bytes;
};

LowpPlan plan(int algo, int64_t n, int64_t k) {
  LowpPlan p{};
  p.nb = (n + KB - 1) / KB;
  p.T = tiles_of(k);
  // BF16X6 on 256 x 128 tiles (one workgroup of 8 waves per CU): 107 -> 97 ms
  // at n = 4e6, k = 2000; BF16X3, which already runs two 4-wave workgroups
  // per CU on 128 x 128 tiles, measured slower on them (61 -> 64 ms)
  const bool wide = algo == DOPINF_GRAM_BF16X6;
  const int T2 = (p.T + 1) / 2;
  p.kp = wide ? int64_t(T2) * 2 * BT : int64_t(p.T) * BT;
  p.ntiles = p.T * (p.T + 1) / 2;
  p.nwide = T2 * (T2 + 1) - (p.T % 2);
  // resident workgroups: two per CU (FP32, BF16X3), one for BF16X6 (8 waves,
  // 144 KB of LDS)
  int slots = 0;
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      slots = (wide ? 1 : 2) * ncu;
  }
  int target = gramplan::choose_splits(n, wide ? p.nwide : p.ntiles, 8192, slots);
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
  pa.vec = (reinterpret_cast<uintptr_t>(Q) % 16 == 0 && ldq % 4 == 0) ? 1 : 0;
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
  pack_kernel<<<dim3(unsigned(p.nb), unsigned(p.kp / BT)), 256, 0, st>>>(pa);
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
  g.sel = 0;
  g.nlaunch = p.ntiles;
  if (algo == DOPINF_GRAM_NATIVE) {
    const int noff = p.T * (p.T - 1) / 2;
    if (noff > 0) {
      g.sel = 1;
      g.nlaunch = noff;
      gram_packed_kernel<0><<<dim3(unsigned(p.nsplit) * unsigned(noff)), NTH, 0, st>>>(g);
      DOPINF_LAUNCHED();
    }
    g.sel = 2;
    g.nlaunch = p.T;
    gram_packed_kernel<0, true><<<dim3(unsigned(p.nsplit) * unsigned(p.T)), NTH, 0, st>>>(g);
  } else if (algo == DOPINF_GRAM_BF16X3) {
    gram_packed_kernel<1><<<grid, NTH, 0, st>>>(g);
  } else {
    WideArgs wa{};
    wa.nb = p.nb;
    wa.kp = p.kp;
    wa.T = p.T;
    wa.nwide = p.nwide;
    wa.nsplit = p.nsplit;
    wa.xcd_map = g.xcd_map;
    wa.bps = p.bps;
    wa.part_p[0] = pa.p0;
    wa.part_p[1] = pa.p1;
    wa.part_p[2] = pa.p2;
    wa.part = g.part;
    gram_wide_kernel<2><<<dim3(unsigned(p.nsplit) * unsigned(p.nwide)), WMT, 0, st>>>(wa);
  }
  DOPINF_LAUNCHED();
  return gram_reduce_launch(st, g.part, p.nsplit, p.ntiles, p.T, 1, k, k, D, ldd);
}
