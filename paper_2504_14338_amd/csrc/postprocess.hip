// Step V of dOpInf (arXiv:2504.14338, Sec. 3.6): the reduced solution mapped
// back to the original coordinates at selected rows, without forming the
// POD basis of all rows.
//
//   V[i, :]    = Qs[row_i, :] T_r                  (rows of V_r, Eq. (7))
//   pred[i, t] = s_v(row_i) (V[i, :] Qtilde[:, t]) + mean[row_i]
//
// Both are products of a tall operand (gathered snapshot rows, or V) with a
// short one (T_r, k x r, or Qtilde, r x N) and run on one FP64 MFMA tile
// kernel: 64 or 128 output rows per workgroup, wave w owns rows 16w..16w+15
// of each 64-row block and NJ blocks of 16 columns; K is staged through LDS
// in chunks of 32 with the next chunk's global loads in registers while the
// current one is used.
// Centering is a subtraction as the snapshot values are staged; the division
// by the variable's scale is applied once per output entry (exact in exact
// arithmetic, and one division per V entry instead of one per Q entry).
#include "common.hpp"

namespace dopinf {
int check_var_rows(int64_t n, int nvars, const int64_t* var_rows_h);

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));

constexpr int PT = 256;   // threads: 4 waves
constexpr int PM = 64;    // output rows per workgroup
constexpr int PK = 32;    // K chunk staged in LDS
// Both stages hold rows of PK = 32 values (A: output rows, B: output
// columns, i.e. B transposed) padded to 34 doubles: the 16 rows x 2 k of a
// half-wave's fragment reads then fall on 64 different 4-byte banks.
constexpr int PAS = PK + 2;

struct VarTable {
  int nvars;
  int64_t row0[DOPINF_MAX_VARS + 1];
};

__device__ __forceinline__ int var_of(const VarTable& vt, int64_t row) {
  int v = 0;
  while (v + 1 < vt.nvars && row >= vt.row0[v + 1]) ++v;
  return v;
}

template <class T>
struct RowGemmArgs {
  const T* A;              // A row i = A[arow(i) * lda + 0 .. K)
  int64_t lda;
  const int64_t* a_rows;   // gather map for A, or null (identity)
  const double* a_shift;   // per source row, subtracted from A's values, or null
  const double* B;         // K x ncol, row-major
  int64_t ldb;
  int64_t m, K, ncol, n_src;
  double* C;               // m x ncol
  int64_t ldc;
  const int64_t* e_rows;   // source row of output row i for the epilogue, or null (identity)
  const double* e_scale;   // per variable: divide (div = 1) or multiply (div = 0), or null
  int div;
  const double* e_add;     // per source row, added after scaling, or null
  VarTable vt;
  int* info;               // receives DOPINF_E_ARG for a row index outside [0, n_src)
};

// RB row blocks of 64 per workgroup: wave w owns rows 16 w + 64 b (b < RB)
// of the tile, so a workgroup reads each chunk of the short operand once for
// 64 RB rows.
template <class T, int NJ, int RB>
__global__ __launch_bounds__(PT) void row_gemm_kernel(RowGemmArgs<T> a) {
  __shared__ double As[PM * RB][PAS];
  __shared__ double Bs[16 * NJ][PAS];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t i0 = int64_t(blockIdx.x) * PM * RB;
  const int64_t c0 = int64_t(blockIdx.y) * 16 * NJ;

  // A staging: thread -> tile rows tid / 4 + 64 b, 8 consecutive k at 8 (tid % 4)
  const int ar = tid >> 2, ak = (tid & 3) * 8;
  int64_t src[RB];
  double shift[RB];
  const T* arow[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const int64_t gi = i0 + ar + PM * b;
    src[b] = -1;
    if (gi < a.m) {
      src[b] = a.a_rows ? a.a_rows[gi] : gi;
      if (src[b] < 0 || src[b] >= a.n_src) {
        if (a.info) atomicExch(a.info, DOPINF_E_ARG);
        src[b] = -1;
      }
    }
    shift[b] = (src[b] >= 0 && a.a_shift) ? a.a_shift[src[b]] : 0.0;
    arow[b] = a.A + (src[b] >= 0 ? src[b] : 0) * a.lda;
  }
  // B staging: thread -> chunk row tid / 8, 2 NJ consecutive columns
  constexpr int BW = 2 * NJ;
  const int br = tid >> 3, bc = (tid & 7) * BW;

  double ra[RB][8], rb[BW];
  // 16-byte loads where a thread's eight A values (or 2 NJ B values) lie
  // inside the matrix and 16-byte aligned; element loads otherwise
  const bool avec = sizeof(T) == 8 && (a.lda % 2) == 0 && (reinterpret_cast<uintptr_t>(a.A) % 16) == 0;
  const bool bvec = (a.ldb % 2) == 0 && (reinterpret_cast<uintptr_t>(a.B) % 16) == 0;
  auto load = [&](int64_t kc) {
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int64_t k0 = kc + ak;
      if (avec && src[b] >= 0 && k0 + 8 <= a.K) {
        const double* p = reinterpret_cast<const double*>(arow[b]) + k0;
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const dbl2 x = *reinterpret_cast<const dbl2*>(p + 2 * h);
          ra[b][2 * h] = x[0] - shift[b];
          ra[b][2 * h + 1] = x[1] - shift[b];
        }
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int64_t kk = k0 + q;
          const bool ok = src[b] >= 0 && kk < a.K;
          const double x = static_cast<double>(arow[b][ok ? kk : 0]);
          ra[b][q] = ok ? x - shift[b] : 0.0;
        }
      }
    }
    const int64_t kb = kc + br;
    if (bvec && kb < a.K && c0 + bc + BW <= a.ncol) {
      const double* p = a.B + kb * a.ldb + c0 + bc;
#pragma unroll
      for (int h = 0; h < BW / 2; ++h) {
        const dbl2 x = *reinterpret_cast<const dbl2*>(p + 2 * h);
        rb[2 * h] = x[0];
        rb[2 * h + 1] = x[1];
      }
    } else {
#pragma unroll
      for (int q = 0; q < BW; ++q) {
        const int64_t c = c0 + bc + q;
        const bool ok = kb < a.K && c < a.ncol;
        const double x = a.B[(ok ? kb : 0) * a.ldb + (ok ? c : 0)];
        rb[q] = ok ? x : 0.0;
      }
    }
  };

  dbl4 acc[RB][NJ];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[b][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  load(0);
  for (int64_t kc = 0; kc < a.K; kc += PK) {
    __syncthreads();  // the previous chunk has been read
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int q = 0; q < 8; ++q) As[ar + PM * b][ak + q] = ra[b][q];
#pragma unroll
    for (int q = 0; q < BW; ++q) Bs[bc + q][br] = rb[q];
    __syncthreads();
    if (kc + PK < a.K) load(kc + PK);
    const int kmax = (a.K - kc) < PK ? int(a.K - kc) : PK;
    for (int kk = 0; kk < kmax; kk += 4) {
      const int k = kk + (lane >> 4);  // rows past K hold zeros
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const double af = As[16 * wv + PM * b + (lane & 15)][k];
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[b][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, Bs[16 * j + (lane & 15)][k], acc[b][j], 0, 0, 0);
      }
    }
  }

  // epilogue: acc[b][j][e] is C[16 wv + 64 b + (lane >> 4) + 4 e][16 j + (lane & 15)]
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = i0 + 16 * wv + PM * b + (lane >> 4) + 4 * e;
      if (i >= a.m) continue;
      const int64_t es = a.e_rows ? a.e_rows[i] : i;
      const bool ok = es >= 0 && es < a.n_src;
      double sc = 1.0, ad = 0.0;
      if (ok) {
        if (a.e_scale) sc = a.e_scale[var_of(a.vt, es)];
        if (a.e_add) ad = a.e_add[es];
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int64_t c = c0 + 16 * j + (lane & 15);
        if (c >= a.ncol) continue;
        double v = acc[b][j][e];
        v = a.div ? v / sc : v * sc;
        a.C[i * a.ldc + c] = ok ? v + ad : NAN;
      }
    }
}

// The basis at all rows (contiguous float64 rows, 33 <= ncol <= 64, even K
// and ncol): both operands go from memory straight into LDS by LDS-DMA
// (buffer loads that write LDS, no register round trip), double buffered in
// stages of 16 values of K, one workgroup barrier per stage, three
// workgroups per CU (48 KB of LDS).  A (128 rows x 16 k, 128 bytes per row)
// is M-major with the eight 16-byte chunks of row m at slots c ^ ((m / 2) % 8),
// so the 16 rows of a fragment read fall on 16 different bank groups; B
// (16 k x 64 columns, 512 bytes per row) is K-major with the chunks of odd
// rows at c ^ 8, so the two k of a fragment read use both halves of the
// banks.  Out-of-range rows, K past its end and columns past ncol read as
// zero (buffer range checks and an out-of-range offset).  The mean is
// subtracted from the A fragments (zero K entries meet zero B entries).
constexpr int DK = 16;                  // K per stage
constexpr int DROWS = 2 * PM;           // output rows per workgroup
constexpr int DA = DROWS * DK;          // doubles of an A stage
constexpr int DB = DK * 64;             // doubles of a B stage
constexpr int DSTAGE = DA + DB;         // 24 KB

#define DOPINF_LDS(p) ((__attribute__((address_space(3))) void*)(p))

__device__ __forceinline__ void wait_vmem_all() { __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8)); }

__device__ __forceinline__ void barrier_only() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

__global__ __launch_bounds__(PT) void row_gemm_dma_kernel(RowGemmArgs<double> a) {
  __shared__ __attribute__((aligned(16))) double sm[2 * DSTAGE];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t i0 = int64_t(blockIdx.x) * DROWS;
  const int64_t mrows = a.m - i0 < DROWS ? a.m - i0 : DROWS;
  const __amdgpu_buffer_rsrc_t rsa =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(a.A + i0 * a.lda), 0, int(mrows * a.lda * 8), 0x00020000);
  const __amdgpu_buffer_rsrc_t rsb =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(a.B), 0, int(a.K * a.ldb * 8), 0x00020000);
  const int64_t nst = (a.K + DK - 1) / DK;
  // wave wv issues the A instructions q = wv + 4 t (8 rows each) and the B
  // instructions q = wv + 4 t (2 k rows each) of a stage
  auto issue = [&](int64_t st) {
    double* S = sm + (st & 1) * DSTAGE;
    const int64_t kb = st * DK;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int q = wv + 4 * t;
      const int m = 8 * q + (lane >> 3);
      const int c = (lane & 7) ^ ((m >> 1) & 7);
      const int64_t k = kb + 2 * c;
      const uint32_t off = (m < mrows && k < a.K) ? uint32_t((int64_t(m) * a.lda + k) * 8) : 0x80000000u;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rsa, DOPINF_LDS(S + q * 128), 16, off, 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int q = wv + 4 * t;
      const int kk = 2 * q + (lane >> 5);
      const int c = (lane & 31) ^ ((kk & 1) << 3);
      const int64_t k = kb + kk;
      const uint32_t off = (k < a.K && 2 * c < a.ncol) ? uint32_t((k * a.ldb + 2 * c) * 8) : 0x80000000u;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rsb, DOPINF_LDS(S + DA + q * 128), 16, off, 0, 0, 0);
    }
  };
  double shift[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int64_t gi = i0 + 16 * wv + PM * b + (lane & 15);
    shift[b] = (a.a_shift && gi < a.m) ? a.a_shift[gi] : 0.0;
  }
  dbl4 acc[2][4];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[b][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  if (nst > 0) issue(0);
  for (int64_t st = 0; st < nst; ++st) {
    wait_vmem_all();
    barrier_only();
    // the other buffer was read in iteration st - 1, which every wave has left
    if (st + 1 < nst) issue(st + 1);
    const double* SA = sm + (st & 1) * DSTAGE;
    const double* SB = SA + DA;
#pragma unroll
    for (int kk = 0; kk < DK / 4; ++kk) {
      const int k = 4 * kk + (lane >> 4);
      double bf[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = 16 * j + (lane & 15);
        bf[j] = SB[k * 64 + 2 * ((col >> 1) ^ ((k & 1) << 3)) + (col & 1)];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int m = 16 * wv + PM * b + (lane & 15);
        const double af = SA[m * DK + 2 * ((k >> 1) ^ ((m >> 1) & 7)) + (k & 1)] - shift[b];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[b][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf[j], acc[b][j], 0, 0, 0);
      }
    }
  }
  // epilogue as in row_gemm_kernel: acc[b][j][e] is C[16 wv + 64 b + (lane >> 4) + 4 e][16 j + (lane & 15)]
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = i0 + 16 * wv + PM * b + (lane >> 4) + 4 * e;
      if (i >= a.m) continue;
      const int64_t es = a.e_rows ? a.e_rows[i] : i;
      const bool ok = es >= 0 && es < a.n_src;
      double sc = 1.0, ad = 0.0;
      if (ok) {
        if (a.e_scale) sc = a.e_scale[var_of(a.vt, es)];
        if (a.e_add) ad = a.e_add[es];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t c = 16 * j + (lane & 15);
        if (c >= a.ncol) continue;
        double v = acc[b][j][e];
        v = a.div ? v / sc : v * sc;
        a.C[i * a.ldc + c] = ok ? v + ad : NAN;
      }
    }
}

// The DMA form applies to contiguous float64 rows of a tall product with
// 33..64 columns, even K and ncol, 16-byte aligned rows and buffer ranges
// below 2 GB.
bool dma_eligible(const RowGemmArgs<double>& a) {
  return !a.a_rows && a.ncol > 32 && a.ncol <= 64 && a.m >= int64_t(256) * DROWS && a.K % 2 == 0 &&
         a.ncol % 2 == 0 && a.lda % 2 == 0 && a.ldb % 2 == 0 && (reinterpret_cast<uintptr_t>(a.A) % 16) == 0 &&
         (reinterpret_cast<uintptr_t>(a.B) % 16) == 0 && int64_t(DROWS) * a.lda * 8 < (int64_t(1) << 31) &&
         a.K * a.ldb * 8 < (int64_t(1) << 31);
}

template <class T, int RB>
void launch_row_gemm_rb(hipStream_t st, const RowGemmArgs<T>& a) {
  const unsigned gx = unsigned((a.m + PM * RB - 1) / (PM * RB));
  if (a.ncol <= 16)
    row_gemm_kernel<T, 1, RB><<<dim3(gx, 1), PT, 0, st>>>(a);
  else if (a.ncol <= 32)
    row_gemm_kernel<T, 2, RB><<<dim3(gx, 1), PT, 0, st>>>(a);
  else if (a.ncol <= 64)
    row_gemm_kernel<T, 4, RB><<<dim3(gx, 1), PT, 0, st>>>(a);
  else
    row_gemm_kernel<T, 8, RB><<<dim3(gx, unsigned((a.ncol + 127) / 128)), PT, 0, st>>>(a);
}

// Tall products (at least 256 row tiles of 128) take 128 rows per
// workgroup; shorter ones 64, for more workgroups.
template <class T>
int launch_row_gemm(hipStream_t st, const RowGemmArgs<T>& a) {
  if constexpr (sizeof(T) == 8) {
    if (dma_eligible(a)) {
      row_gemm_dma_kernel<<<unsigned((a.m + DROWS - 1) / DROWS), PT, 0, st>>>(a);
      DOPINF_LAUNCHED();
      return DOPINF_OK;
    }
  }
  if (a.m >= int64_t(256) * 2 * PM)
    launch_row_gemm_rb<T, 2>(st, a);
  else
    launch_row_gemm_rb<T, 1>(st, a);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}

__global__ void set_int_kernel(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

template <class T>
int postprocess_t(hipStream_t st, const T* Q, int64_t n, int64_t k, int64_t ldq, const double* mean,
                  const double* scale, const VarTable& vt, const int64_t* rows, int64_t m, const double* Tr,
                  int64_t ldtr, int r, const double* Qtilde, int64_t ldqt, int64_t n_out, double* V, int64_t ldv,
                  double* pred, int64_t ldp, int* info) {
  RowGemmArgs<T> b{};
  b.A = Q;
  b.lda = ldq;
  b.a_rows = rows;
  b.a_shift = mean;
  b.B = Tr;
  b.ldb = ldtr;
  b.m = m;
  b.K = k;
  b.ncol = r;
  b.n_src = n;
  b.C = V;
  b.ldc = ldv;
  b.e_rows = rows;
  b.e_scale = scale;
  b.div = 1;
  b.e_add = nullptr;
  b.vt = vt;
  b.info = info;
  int rc = launch_row_gemm(st, b);
  if (rc || !pred) return rc;
  RowGemmArgs<double> p{};
  p.A = V;
  p.lda = ldv;
  p.a_rows = nullptr;
  p.a_shift = nullptr;
  p.B = Qtilde;
  p.ldb = ldqt;
  p.m = m;
  p.K = r;
  p.ncol = n_out;
  p.n_src = n;
  p.C = pred;
  p.ldc = ldp;
  p.e_rows = rows;
  p.e_scale = scale;
  p.div = 0;
  p.e_add = mean;
  p.vt = vt;
  p.info = nullptr;
  return launch_row_gemm(st, p);
}

}  // namespace

// C (m x ncol) = A (m x K) B (K x ncol), all row-major float64: the same tile
// kernel, for other parts of the library.
int row_gemm_f64(hipStream_t st, const double* A, int64_t lda, int64_t m, int64_t K, const double* B, int64_t ldb,
                 int64_t ncol, double* C, int64_t ldc) {
  RowGemmArgs<double> g{};
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.ldb = ldb;
  g.m = m;
  g.K = K;
  g.ncol = ncol;
  g.n_src = m;
  g.C = C;
  g.ldc = ldc;
  g.div = 0;
  g.vt.nvars = 1;
  g.vt.row0[0] = 0;
  g.vt.row0[1] = m;
  return launch_row_gemm(st, g);
}

}  // namespace dopinf

using namespace dopinf;

extern "C" int dopinf_postprocess(void* stream, int dtype, const void* Q, int64_t n, int64_t k, int64_t ldq,
                                  const double* mean, const double* scale, int nvars, const int64_t* var_rows_h,
                                  const int64_t* rows, int64_t m, const double* Tr, int64_t ldtr, int r,
                                  const double* Qtilde, int64_t ldqt, int64_t n_out, double* V, int64_t ldv,
                                  double* pred, int64_t ldp, int* info) {
  DOPINF_REQUIRE(dtype == DOPINF_F64 || dtype == DOPINF_F32, "dtype must be DOPINF_F64 or DOPINF_F32");
  DOPINF_REQUIRE(Q && Tr && V, "Q, Tr and V must be non-NULL");
  DOPINF_REQUIRE(n >= 1 && k >= 1 && ldq >= k, "need n >= 1, k >= 1, ldq >= k");
  DOPINF_REQUIRE(m >= 1 && (rows || m <= n), "need m >= 1 (and m <= n when rows is NULL)");
  DOPINF_REQUIRE(r >= 1 && r <= k && ldtr >= r, "need 1 <= r <= k and ldtr >= r");
  DOPINF_REQUIRE(ldv >= r, "need ldv >= r");
  if (pred) {
    DOPINF_REQUIRE(Qtilde && n_out >= 1 && ldqt >= n_out && ldp >= n_out,
                   "pred needs Qtilde, n_out >= 1, ldqt >= n_out and ldp >= n_out");
  }
  VarTable vt{};
  vt.nvars = 1;
  vt.row0[0] = 0;
  vt.row0[1] = n;
  if (scale) {
    const int rc = check_var_rows(n, nvars, var_rows_h);
    if (rc) return rc;
    vt.nvars = nvars;
    for (int v = 0; v <= nvars; ++v) vt.row0[v] = var_rows_h[v];
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (info) {
    set_int_kernel<<<1, 64, 0, st>>>(info, DOPINF_OK);
    DOPINF_LAUNCHED();
  }
  if (dtype == DOPINF_F64)
    return postprocess_t(st, static_cast<const double*>(Q), n, k, ldq, mean, scale, vt, rows, m, Tr, ldtr, r,
                         Qtilde, ldqt, n_out, V, ldv, pred, ldp, info);
  return postprocess_t(st, static_cast<const float*>(Q), n, k, ldq, mean, scale, vt, rows, m, Tr, ldtr, r, Qtilde,
                       ldqt, n_out, V, ldv, pred, ldp, info);
}
