// Step III of dOpInf (arXiv:2504.14338, Sec. 3.4): the Gram matrix
// D = Qs^T Qs of a tall-skinny snapshot matrix (Eq. (5)), and the cross Gram
// X^T Y used to project snapshots through Eq. (8).
//
// Design (gfx950):
//  * D is cut into 128 x 128 tiles; only the lower triangle of tiles is
//    computed (symmetry) and mirrored by the reduction.
//  * The n rows are cut into splits (split-K).  Splits never straddle a state
//    variable, so one scale factor 1/s_v^2 applies to a whole partial tile.
//    One workgroup = (tile, split); the grid holds ~8k workgroups so the 256
//    CUs see ~15 rounds of work and a small tail.
//  * Workgroup: 4 waves in a 2 x 2 arrangement, each owning a 64 x 64
//    sub-tile = 4 x 4 blocks of v_mfma_f64_16x16x4 (FP64 accumulate).  The
//    symmetric Gram runs the tiles below the diagonal in one launch (whole
//    rounds of resident workgroups) and the diagonal tiles in a second one,
//    where each wave computes 9 of the 36 lower 16 x 16 blocks.
//  * Main kernel (rows 16-byte aligned): panel rows go from HBM straight into
//    LDS with buffer loads in LDS-DMA mode (no register staging).  A buffer
//    descriptor spans one row, so columns past the row and rows past the split
//    read as zero; the per-row temporal means travel the same way.  Two LDS
//    stages of 16 rows; the loads of stage s+1 are in flight while stage s
//    feeds the matrix cores.  Centering (x - mean_i) is applied to the
//    fragments as they leave LDS, so Q is read as stored and never rewritten.
//    75.8 KB of LDS per workgroup: two workgroups share a CU.
//  * Fallback kernel (any alignment): the same tiling with register-staged
//    loads, centering and scaling applied while staging.
//  * XCD-aware order: consecutive workgroup ids go round-robin to the 8 XCDs;
//    ids are mapped so that each XCD walks through its own splits with all
//    tiles of a split together, i.e. the tiles running on one XCD share the
//    same rows and re-read them from that XCD's L2.
//  * Each (tile, split) writes its partial tile to the workspace; a second
//    kernel sums the partials in fixed split order (deterministic, no float
//    atomics) and writes both triangles.
#include "common.hpp"
#include "gram_plan.hpp"

namespace dopinf {
int check_var_rows(int64_t n, int nvars, const int64_t* var_rows_h);

namespace {

using gramplan::SplitPlan;
using gramplan::choose_splits;

// Resident workgroups of the FP64 Gram kernels on the current device (two
// per CU; 0 if the device cannot be queried).
int gram_slots() {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return 2 * ncu;
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int BT = 128;     // tile edge
constexpr int NTH = 256;    // threads per workgroup
constexpr int KC = 16;      // rows per LDS stage (FP64)
constexpr int PAD = 2;      // LDS row padding (doubles)
constexpr int LDR = BT + PAD;

struct GramArgs {
  const double* X;
  int64_t ldx;
  const double* Y;
  int64_t ldy;
  int64_t mx, my;
  int tiles_y;     // tiles along Y (rectangular mode)
  int ntiles;
  int triangle;    // X == Y: lower triangle of tiles only
  int sel;         // tiles of an LDS-DMA launch: 0 all, 1 below the diagonal, 2 on it
  int nlaunch;     // tiles per split in that launch
  const double* mean;   // may be null
  const double* scale;  // may be null
  double* part;
};

__device__ __forceinline__ void tile_coords(const GramArgs& g, int t, int& I, int& J) {
  if (g.triangle) {
    gramplan::tri_coords(t, I, J);
  } else {
    I = t / g.tiles_y;
    J = t % g.tiles_y;
  }
}

// Load 8 consecutive doubles of one panel row into registers, transformed.
__device__ __forceinline__ void load_row8(const double* __restrict__ P, int64_t ld, int64_t row, int64_t hi,
                                          int64_t col, int64_t mcols, bool vec_ok, double mu, double inv,
                                          bool xf, double (&r)[8]) {
  if (row < hi) {
    const double* p = P + row * ld + col;
    if (vec_ok && col + 8 <= mcols) {
      const double2* p2 = reinterpret_cast<const double2*>(p);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        double2 w = p2[u];
        r[2 * u] = w.x;
        r[2 * u + 1] = w.y;
      }
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) r[u] = (col + u < mcols) ? p[u] : 0.0;
    }
    if (xf) {
#pragma unroll
      for (int u = 0; u < 8; ++u) r[u] = (col + u < mcols) ? (r[u] - mu) * inv : 0.0;
    }
  } else {
#pragma unroll
    for (int u = 0; u < 8; ++u) r[u] = 0.0;
  }
}

__global__ __launch_bounds__(NTH, 2) void gram_f64_mfma_kernel(GramArgs g, SplitPlan sp) {
  __shared__ double As[2][KC][LDR];
  __shared__ double Bs[2][KC][LDR];

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
  tile_coords(g, t, I, J);
  int64_t lo, hi;
  int v;
  gramplan::split_range(sp, s, KC, lo, hi, v);
  const bool diag = g.triangle && (I == J);
  const int64_t a0 = int64_t(I) * BT, b0 = int64_t(J) * BT;
  const bool xf = (g.mean != nullptr) || (g.scale != nullptr);
  const double inv = g.scale ? 1.0 / g.scale[v] : 1.0;
  const bool vecx = ((g.ldx & 1) == 0) && ((reinterpret_cast<uintptr_t>(g.X) & 15) == 0);
  const bool vecy = ((g.ldy & 1) == 0) && ((reinterpret_cast<uintptr_t>(g.Y) & 15) == 0);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int lrow = tid >> 4;          // staging: panel row 0..15
  const int lcol = (tid & 15) * 8;    // staging: first of 8 columns

  dbl4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  const int64_t nst = (hi - lo + KC - 1) / KC;
  double ra[8], rb[8];

  auto fetch = [&](int64_t st) {
    const int64_t row = lo + st * KC + lrow;
    const double mu = (g.mean && row < hi) ? g.mean[row] : 0.0;
    load_row8(g.X, g.ldx, row, hi, a0 + lcol, g.mx, vecx, mu, inv, xf, ra);
    if (!diag) load_row8(g.Y, g.ldy, row, hi, b0 + lcol, g.my, vecy, mu, inv, xf, rb);
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 8; ++u) As[buf][lrow][lcol + u] = ra[u];
    if (!diag) {
#pragma unroll
      for (int u = 0; u < 8; ++u) Bs[buf][lrow][lcol + u] = rb[u];
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
    const double(*Bp)[LDR] = diag ? As[buf] : Bs[buf];
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const int krow = kk * 4 + (lane >> 4);
      const int cm = lane & 15;
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[buf][krow][wm * 64 + i * 16 + cm];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bp[krow][wn * 64 + j * 16 + cm];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (st + 1 < nst) stash(buf ^ 1);
    __syncthreads();
  }

  // partial tile: row index from X's column block, column index from Y's
  double* out = g.part + (size_t(s) * g.ntiles + t) * (BT * BT);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // v_mfma_f64_16x16x4: lane l, element e holds row (l / 16) + 4 e, column l % 16
        const int rr = wm * 64 + i * 16 + (lane >> 4) + 4 * e;
        const int cc = wn * 64 + j * 16 + (lane & 15);
        out[rr * BT + cc] = acc[i][j][e];
      }
}

// ---- LDS-DMA kernel ---------------------------------------------------------

constexpr int DKC = 16;                          // rows per LDS stage
constexpr int DPD = 144;                         // LDS row pitch (doubles)
constexpr int DSLOT = 2 * DKC * DPD + 4 * 32;    // A rows, B rows, 32 means per wave
constexpr int DRPW = DKC / 4;                    // panel rows loaded per wave per stage

#define DOPINF_LDS(p) ((__attribute__((address_space(3))) void*)(p))

// Buffer descriptor over [p, p + nbytes): reads past nbytes return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t span_rsrc(const void* p, int64_t nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, int(nbytes), 0x00020000);
}

// Wait until at most N vector-memory operations of this wave are in flight.
template <int N>
__device__ __forceinline__ void wait_vmem() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Workgroup barrier that does not drain outstanding LDS-DMA loads (the
// explicit wait above decides what must have landed).
__device__ __forceinline__ void barrier_only() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Blocks of 16 x 16 computed by wave w (0..3) of a diagonal tile: the 9
// blocks p = 0..8 of block columns w (block rows w..7) and 7 - w (block rows
// 7 - w..7), which cover the tile's lower triangle of 8 x 8 blocks (36) with
// 9 per wave.  Accumulator p is acc[p / 4][p % 4].
__device__ __forceinline__ void diag_block(int w, int p, int& br, int& bc) {
  const bool first = p < 8 - w;
  br = first ? w + p : p - 1;
  bc = first ? w : 7 - w;
}

// One k-step of wave W of a diagonal tile: block columns W (block rows
// W..7) and 7 - W (block rows 7 - W..7, a subset of the former), so the
// fragments of rows W..7 are read once and serve both columns; accumulator
// p = diag_block's index.  Ak points at (k-row, lane column) of the panel.
template <int W>
__device__ __forceinline__ void diag_step(const double* Ak, double mu, dbl4 (&acc)[4][4]) {
  double af[8 - W];
#pragma unroll
  for (int i = 0; i < 8 - W; ++i) af[i] = Ak[(W + i) * 16] - mu;  // block row W + i (also column W + i)
  const double b_lo = af[0];                                     // column W
  const double b_hi = af[7 - 2 * W];                             // column 7 - W
#pragma unroll
  for (int p = 0; p < 8 - W; ++p)  // (W + p, W)
    acc[p >> 2][p & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[p], b_lo, acc[p >> 2][p & 3], 0, 0, 0);
#pragma unroll
  for (int q = 0; q <= W; ++q) {  // (7 - W + q, 7 - W), p = 8 - W + q
    const int p = 8 - W + q;
    acc[p >> 2][p & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[7 - 2 * W + q], b_hi, acc[p >> 2][p & 3], 0, 0, 0);
  }
}

template <bool DIAG, bool XF>
__device__ __forceinline__ void dma_tile(const GramArgs& g, int64_t lo, int64_t hi, int64_t a0, int64_t b0, double* lds,
                                         dbl4 (&acc)[4][4]) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int wm = w >> 1, wn = w & 1;
  const int64_t nst = (hi - lo + DKC - 1) / DKC;
  const uint32_t offa = uint32_t((a0 + 2 * lane) * 8);
  const uint32_t offb = uint32_t((b0 + 2 * lane) * 8);
  const uint32_t offm = uint32_t(lane) * 4;
  const int64_t bytes_x = g.ldx * 8, bytes_y = g.ldy * 8;

  auto issue = [&](int64_t st) {
    double* sl = lds + (st & 1) * DSLOT;
    const int64_t r0 = lo + st * DKC;
#pragma unroll
    for (int q = 0; q < DRPW; ++q) {
      const int r = w * DRPW + q;
      const int64_t row = r0 + r;
      const bool in = row < hi;
      const int64_t rr = in ? row : lo;
      const __amdgpu_buffer_rsrc_t ra = span_rsrc(g.X + rr * g.ldx, in ? bytes_x : 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, DOPINF_LDS(sl + r * DPD), 16, offa, 0, 0, 0);
      if (!DIAG) {
        const __amdgpu_buffer_rsrc_t rb = span_rsrc(g.Y + rr * g.ldy, in ? bytes_y : 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, DOPINF_LDS(sl + (DKC + r) * DPD), 16, offb, 0, 0, 0);
      }
    }
    if (XF) {
      // lane l brings half of mean[r0 + l / 2]; rows past the split read as 0
      const int64_t nm = (hi - r0) < 32 ? (hi - r0) : 32;
      const __amdgpu_buffer_rsrc_t rmu = span_rsrc(g.mean + r0, nm * 8);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rmu, DOPINF_LDS(sl + 2 * DKC * DPD + w * 32), 4, offm, 0, 0, 0);
    }
  };


  if (nst > 0) issue(0);
  for (int64_t st = 0; st < nst; ++st) {
    wait_vmem<0>();
    barrier_only();
    if (st + 1 < nst) issue(st + 1);
    const double* sl = lds + (st & 1) * DSLOT;
    const double* As = sl;
    const double* Bs = DIAG ? sl : sl + DKC * DPD;
    const double* Ms = sl + 2 * DKC * DPD + w * 32;
#pragma unroll
    for (int kk = 0; kk < DKC / 4; ++kk) {
      const int krow = kk * 4 + (lane >> 4);
      const int cm = lane & 15;
      const double mu = XF ? Ms[krow] : 0.0;
      if (DIAG) {
        // the 9 lower blocks of wave w (diag_block), with w a constant in
        // each branch (w is wave-uniform)
        const double* Ak = As + krow * DPD + cm;
        switch (w) {
          case 0: diag_step<0>(Ak, mu, acc); break;
          case 1: diag_step<1>(Ak, mu, acc); break;
          case 2: diag_step<2>(Ak, mu, acc); break;
          default: diag_step<3>(Ak, mu, acc); break;
        }
      } else {
        double af[4], bf[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) af[i] = As[krow * DPD + wm * 64 + i * 16 + cm] - mu;
#pragma unroll
        for (int j = 0; j < 4; ++j) bf[j] = Bs[krow * DPD + wn * 64 + j * 16 + cm] - mu;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    }
  }
}

// One launch covers the tiles that g.sel selects: all of a rectangular
// Gram, or, for the symmetric one, the tiles below the diagonal (DIAG false)
// and then the diagonal tiles (DIAG true) in a launch of their own.  A
// diagonal tile needs 36 of its 64 blocks, 9 per wave; in the launch of the
// full tiles its workgroups would finish early and leave the rounds of
// resident workgroups ragged, in a launch of their own they fill rounds of
// equal work.
template <bool DIAG>
__global__ __launch_bounds__(NTH, 2) void gram_f64_dma_kernel(GramArgs g, SplitPlan sp) {
  __shared__ double lds[2 * DSLOT];
  int tl, s;
  {
    const int bid = blockIdx.x;
    if (sp.xcd_map) {
      const int xcd = bid & 7;
      const int local = bid >> 3;
      s = (local / g.nlaunch) * 8 + xcd;
      tl = local % g.nlaunch;
    } else {
      s = bid / g.nlaunch;
      tl = bid % g.nlaunch;
    }
  }
  int I, J, t;  // tile coordinates and index of the partial tile
  if (g.sel == 1) {
    gramplan::tri_coords(tl, I, J);  // tl-th tile strictly below: (I + 1, J)
    ++I;
    t = I * (I + 1) / 2 + J;
  } else if (g.sel == 2) {
    I = J = tl;
    t = I * (I + 1) / 2 + I;
  } else {
    tile_coords(g, tl, I, J);
    t = tl;
  }
  int64_t lo, hi;
  int v;
  gramplan::split_range(sp, s, DKC, lo, hi, v);
  const int64_t a0 = int64_t(I) * BT, b0 = int64_t(J) * BT;

  dbl4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  if (g.mean)
    dma_tile<DIAG, true>(g, lo, hi, a0, b0, lds, acc);
  else
    dma_tile<DIAG, false>(g, lo, hi, a0, b0, lds, acc);

  // both operands carry 1/s_v: the partial tile takes 1/s_v^2
  double f = 1.0;
  if (g.scale) {
    const double sv = g.scale[v];
    f = 1.0 / (sv * sv);
  }
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1;
  double* out = g.part + (size_t(s) * g.ntiles + t) * (BT * BT);
  // v_mfma_f64_16x16x4: lane l, element e holds row (l / 16) + 4 e, column
  // l % 16 of a 16 x 16 block.  A diagonal tile writes its lower blocks only
  // (the reduction reads nothing above the diagonal).
  if (DIAG) {
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      int br, bc;
      diag_block(w, p, br, bc);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = br * 16 + (lane >> 4) + 4 * e;
        const int cc = bc * 16 + (lane & 15);
        out[rr * BT + cc] = acc[p >> 2][p & 3][e] * f;
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = wm * 64 + i * 16 + (lane >> 4) + 4 * e;
        const int cc = wn * 64 + j * 16 + (lane & 15);
        out[rr * BT + cc] = acc[i][j][e] * f;
      }
}

// The LDS-DMA kernel needs 16-byte aligned rows and descriptor-sized row spans.
bool dma_ok(const double* P, int64_t ld) {
  return (reinterpret_cast<uintptr_t>(P) & 15) == 0 && (ld & 1) == 0 && ld * 8 < (int64_t(1) << 31);
}

// Sum partial tiles over splits in fixed order and write C (both triangles
// for the symmetric case).
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* __restrict__ part, int nsplit,
                                                          int ntiles, int tiles_y, int triangle, int64_t mx,
                                                          int64_t my, double* __restrict__ C, int64_t ldc) {
  const int t = blockIdx.x;
  const int rr = blockIdx.y * 2 + (threadIdx.x >> 7);
  const int cc = threadIdx.x & 127;
  int I, J;
  if (triangle) {
    gramplan::tri_coords(t, I, J);
  } else {
    I = t / tiles_y;
    J = t % tiles_y;
  }
  const int64_t a = int64_t(I) * BT + rr, b = int64_t(J) * BT + cc;
  if (a >= mx || b >= my) return;
  if (triangle && I == J && rr < cc) return;
  double sum = 0.0;
  const size_t stride = size_t(ntiles) * BT * BT;
  const double* p = part + size_t(t) * BT * BT + size_t(rr) * BT + cc;
  for (int s = 0; s < nsplit; ++s) sum += p[s * stride];
  C[a * ldc + b] = sum;
  if (triangle) C[b * ldc + a] = sum;
}

int tiles_of(int64_t m) { return int((m + BT - 1) / BT); }

size_t part_bytes(int nsplit, int ntiles) { return size_t(nsplit) * ntiles * BT * BT * sizeof(double); }

int run_gram(hipStream_t st, GramArgs g, const SplitPlan& sp, double* C, int64_t ldc, int tiles_y) {
  g.tiles_y = tiles_y;
  dim3 grid(unsigned(sp.nsplit) * unsigned(g.ntiles));
  if (dma_ok(g.X, g.ldx) && dma_ok(g.Y, g.ldy)) {
    if (g.triangle) {
      const int noff = tiles_y * (tiles_y - 1) / 2;
      if (noff > 0) {
        g.sel = 1;
        g.nlaunch = noff;
        gram_f64_dma_kernel<false><<<dim3(unsigned(sp.nsplit) * unsigned(noff)), NTH, 0, st>>>(g, sp);
        DOPINF_LAUNCHED();
      }
      g.sel = 2;
      g.nlaunch = tiles_y;
      gram_f64_dma_kernel<true><<<dim3(unsigned(sp.nsplit) * unsigned(tiles_y)), NTH, 0, st>>>(g, sp);
    } else {
      g.sel = 0;
      g.nlaunch = g.ntiles;
      gram_f64_dma_kernel<false><<<grid, NTH, 0, st>>>(g, sp);
    }
  } else {
    gram_f64_mfma_kernel<<<grid, NTH, 0, st>>>(g, sp);
  }
  DOPINF_LAUNCHED();
  dim3 rgrid(unsigned(g.ntiles), BT / 2);
  gram_reduce_kernel<<<rgrid, 256, 0, st>>>(g.part, sp.nsplit, g.ntiles, tiles_y, g.triangle, g.mx, g.my, C, ldc);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}

}  // namespace

int gram_reduce_launch(hipStream_t st, const double* part, int nsplit, int ntiles, int tiles_y, int triangle,
                       int64_t mx, int64_t my, double* C, int64_t ldc) {
  dim3 rgrid(unsigned(ntiles), BT / 2);
  gram_reduce_kernel<<<rgrid, 256, 0, st>>>(part, nsplit, ntiles, tiles_y, triangle, mx, my, C, ldc);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}

// Symmetric Gram of an n x m float64 matrix (used by Step IV's data Gram as
// well): D = Xs^T Xs with the optional per-row / per-variable transform.
int gram_f64_internal(hipStream_t st, const double* X, int64_t n, int64_t m, int64_t ldx, const double* mean,
                      const double* scale, int nvars, const int64_t* var_rows_h, double* D, int64_t ldd,
                      void* ws, size_t ws_bytes) {
  const int T = tiles_of(m);
  const int ntiles = T * (T + 1) / 2;
  int64_t one_var[2] = {0, n};
  if (!var_rows_h) {
    nvars = 1;
    var_rows_h = one_var;
  }
  SplitPlan sp = gramplan::make_plan(n, nvars, var_rows_h, choose_splits(n, ntiles, 8192, gram_slots()), KC);
  if (ws_bytes < part_bytes(sp.nsplit, ntiles) || !ws)
    return fail(DOPINF_E_WORKSPACE, "gram workspace of %zu bytes needed, %zu given", part_bytes(sp.nsplit, ntiles),
                ws_bytes);
  GramArgs g{};
  g.X = X;
  g.ldx = ldx;
  g.Y = X;
  g.ldy = ldx;
  g.mx = m;
  g.my = m;
  g.ntiles = ntiles;
  g.triangle = 1;
  g.mean = mean;
  g.scale = scale;
  g.part = static_cast<double*>(ws);
  return run_gram(st, g, sp, D, ldd, T);
}

size_t gram_f64_workspace_internal(int64_t n, int64_t m, int nvars) {
  const int T = tiles_of(m);
  const int ntiles = T * (T + 1) / 2;
  // per-variable rounding can add at most nvars splits
  return part_bytes(choose_splits(n, ntiles, 8192, gram_slots()) + nvars + 8, ntiles);
}

}  // namespace dopinf

using namespace dopinf;

namespace dopinf {
size_t cross_gram_workspace_internal(int64_t n, int64_t mx, int64_t my);
size_t gram_i8_workspace(int64_t n, int64_t k);
int gram_i8(hipStream_t st, const float* Q, int64_t n, int64_t k, int64_t ldq, const double* mean,
            const double* scale, int nvars, const int64_t* var_rows_h, double* D, int64_t ldd, void* ws,
            size_t ws_bytes);
}

size_t gram_lowp_workspace(int algo, int64_t n, int64_t k);
int gram_lowp(hipStream_t st, int algo, const float* Q, int64_t n, int64_t k, int64_t ldq, const double* mean,
              const double* scale, int nvars, const int64_t* var_rows_h, double* D, int64_t ldd, void* ws,
              size_t ws_bytes);

extern "C" size_t dopinf_gram_workspace(int dtype, int algo, int64_t n, int64_t k) {
  if (n <= 0 || k <= 0) return 0;
  if (dtype == DOPINF_F64) return gram_f64_workspace_internal(n, k, DOPINF_MAX_VARS);
  if (algo == DOPINF_GRAM_I8X6) return gram_i8_workspace(n, k);
  return gram_lowp_workspace(algo, n, k);
}

extern "C" int dopinf_gram(void* stream, int dtype, int algo, const void* Q, int64_t n, int64_t k, int64_t ldq,
                           const double* mean, const double* scale, int nvars, const int64_t* var_rows_h,
                           double* D, int64_t ldd, void* ws, size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  DOPINF_REQUIRE(Q && D, "Q and D must be non-NULL");
  DOPINF_REQUIRE(n >= 1 && k >= 1 && ldq >= k && ldd >= k, "need n >= 1, k >= 1, ldq >= k, ldd >= k");
  DOPINF_REQUIRE(k <= (int64_t(1) << 20), "k too large");
  if (scale) {
    int rc = check_var_rows(n, nvars, var_rows_h);
    if (rc) return rc;
  } else if (var_rows_h) {
    int rc = check_var_rows(n, nvars, var_rows_h);
    if (rc) return rc;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == DOPINF_F64) {
    DOPINF_REQUIRE(algo == DOPINF_GRAM_NATIVE, "float64 data supports DOPINF_GRAM_NATIVE only");
    return gram_f64_internal(st, static_cast<const double*>(Q), n, k, ldq, mean, scale, scale ? nvars : 0,
                             scale ? var_rows_h : nullptr, D, ldd, ws, ws_bytes);
  }
  DOPINF_REQUIRE(dtype == DOPINF_F32, "dtype must be DOPINF_F64 or DOPINF_F32");
  DOPINF_REQUIRE(algo == DOPINF_GRAM_NATIVE || algo == DOPINF_GRAM_BF16X3 || algo == DOPINF_GRAM_BF16X6 ||
                     algo == DOPINF_GRAM_I8X6,
                 "unknown gram algorithm");
  if (algo == DOPINF_GRAM_I8X6)
    return gram_i8(st, static_cast<const float*>(Q), n, k, ldq, mean, scale, scale ? nvars : 0,
                   scale ? var_rows_h : nullptr, D, ldd, ws, ws_bytes);
  return gram_lowp(st, algo, static_cast<const float*>(Q), n, k, ldq, mean, scale, scale ? nvars : 0,
                   scale ? var_rows_h : nullptr, D, ldd, ws, ws_bytes);
}

extern "C" size_t dopinf_cross_gram_workspace(int64_t n, int64_t mx, int64_t my) {
  if (n <= 0 || mx <= 0 || my <= 0) return 0;
  return cross_gram_workspace_internal(n, mx, my);
}

namespace dopinf {

int cross_gram_internal(hipStream_t st, const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n,
                        int64_t mx, int64_t my, double* C, int64_t ldc, void* ws, size_t ws_bytes,
                        const double* mean, const double* scale, int nvars, const int64_t* var_rows_h) {
  const int ty = tiles_of(my);
  const int ntiles = tiles_of(mx) * ty;
  int64_t one_var[2] = {0, n};
  if (!var_rows_h || nvars < 1) {
    nvars = 1;
    var_rows_h = one_var;
  }
  SplitPlan sp = gramplan::make_plan(n, nvars, var_rows_h, choose_splits(n, ntiles, 8192, gram_slots()), KC);
  if (!ws || ws_bytes < part_bytes(sp.nsplit, ntiles))
    return fail(DOPINF_E_WORKSPACE, "cross gram workspace of %zu bytes needed, %zu given",
                part_bytes(sp.nsplit, ntiles), ws_bytes);
  GramArgs g{};
  g.X = X;
  g.ldx = ldx;
  g.Y = Y;
  g.ldy = ldy;
  g.mx = mx;
  g.my = my;
  g.ntiles = ntiles;
  g.triangle = 0;
  g.mean = mean;
  g.scale = scale;
  g.part = static_cast<double*>(ws);
  return run_gram(st, g, sp, C, ldc, ty);
}

size_t cross_gram_workspace_internal(int64_t n, int64_t mx, int64_t my) {
  const int ntiles = tiles_of(mx) * tiles_of(my);
  return part_bytes(choose_splits(n, ntiles, 8192, gram_slots()) + DOPINF_MAX_VARS + 8, ntiles);
}

}  // namespace dopinf

extern "C" int dopinf_cross_gram(void* stream, const double* X, int64_t ldx, const double* Y, int64_t ldy,
                                 int64_t n, int64_t mx, int64_t my, const double* mean, const double* scale,
                                 int nvars, const int64_t* var_rows_h, double* C, int64_t ldc, void* ws,
                                 size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  DOPINF_REQUIRE(X && Y && C, "X, Y and C must be non-NULL");
  DOPINF_REQUIRE(n >= 1 && mx >= 1 && my >= 1 && ldx >= mx && ldy >= my && ldc >= my,
                 "need n, mx, my >= 1 and ldx >= mx, ldy >= my, ldc >= my");
  if (scale || var_rows_h) {
    int rc = check_var_rows(n, nvars, var_rows_h);
    if (rc) return rc;
  }
  return cross_gram_internal(static_cast<hipStream_t>(stream), X, ldx, Y, ldy, n, mx, my, C, ldc, ws, ws_bytes,
                             mean, scale, scale ? nvars : 0, scale ? var_rows_h : nullptr);
}
