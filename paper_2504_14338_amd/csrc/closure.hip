// Learned closure for the discrete quadratic ROM of Eq. (11) (arXiv:2504.14338
// gives the ROM; the closure is an addition of this library):
//   q_{t+1} = f_ROM(q_t) + g(q_t),   g: R^r -> R^r, r -> 128 -> 128 -> r, GELU,
// trained on the ROM's one-step residuals of the reduced training data.
//
// Arithmetic: standardized inputs, weights and hidden activations are rounded
// to bfloat16 (round to nearest even) before each product; products and sums
// are float32 (bf16 x bf16 products are exact in float32); biases, master
// weights and Adam state are float32; the ROM part is float64.
//
// Kernels:
//  * residual_kernel      rho_t = qhat_{t+1} - f_ROM(qhat_t)
//  * norm_kernel          per-mode mean / population std of inputs and targets
//  * train_kernel         ONE persistent workgroup of 8 waves runs every
//                         epoch on the matrix cores: per minibatch forward,
//                         backward and weight gradients in chunks of 32 rows,
//                         Adam applied by the lanes that own each gradient.
//  * grad_kernel          the same forward/backward over one batch (gradient
//                         checks)
//  * eval_kernel          g(x) for a batch of states and max ||g||
//  * closure_rollout_kernel  4 rollouts per workgroup: MLP and ROM per step,
//                         latched fallback to the plain ROM when ||g|| exceeds
//                         the threshold, growth / error / finiteness scores.
#include "common.hpp"
#include "xwg_sync.hpp"

namespace dopinf {
namespace {

constexpr int H = 128;       // hidden width
constexpr int BMAX = 256;    // largest minibatch
constexpr int RG = 16;       // rollouts (or eval rows) per workgroup
constexpr int ET = 256;      // eval / rollout threads

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

__host__ __device__ inline int64_t nquad(int64_t r) { return r * (r + 1) / 2; }
__host__ __device__ inline int64_t ncols(int64_t r) { return r + nquad(r) + 1; }

struct Off {
  int64_t w1, b1, w2, b2, w3, b3, P;
  __host__ __device__ explicit Off(int r) {
    w1 = 0;
    b1 = int64_t(H) * r;
    w2 = b1 + H;
    b2 = w2 + int64_t(H) * H;
    w3 = b2 + H;
    b3 = w3 + int64_t(r) * H;
    P = b3 + r;
  }
};

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return static_cast<unsigned short>((u >> 16) | 0x40);
  const unsigned int lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return static_cast<unsigned short>(u >> 16);
}
__device__ __forceinline__ float bf16f(float f) { return __uint_as_float(unsigned(bf16_bits(f)) << 16); }
__device__ __forceinline__ float wb(const unsigned short* W, int64_t i) { return __uint_as_float(unsigned(W[i]) << 16); }
__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// bf16 copies of the three weight matrices: [W1 (H x r) | W2 (H x H) | W3 (r x H)]
__device__ void load_wb(const float* __restrict__ p, int r, unsigned short* Wb, int tid, int nt) {
  const Off o(r);
  const int64_t n1 = int64_t(H) * r, n2 = int64_t(H) * H, n3 = int64_t(r) * H;
  for (int64_t e = tid; e < n1; e += nt) Wb[e] = bf16_bits(p[o.w1 + e]);
  for (int64_t e = tid; e < n2; e += nt) Wb[n1 + e] = bf16_bits(p[o.w2 + e]);
  for (int64_t e = tid; e < n3; e += nt) Wb[n1 + n2 + e] = bf16_bits(p[o.w3 + e]);
}

// forward for R rows of standardized bf16-valued inputs x (R x r)
template <int NT>
__device__ void mlp_fwd(int R, int r, const unsigned short* Wb, const float* __restrict__ p, const float* x, float* z1,
                        float* a1, float* z2, float* a2, float* out, int tid) {
  const Off o(r);
  const unsigned short* W1 = Wb;
  const unsigned short* W2 = Wb + int64_t(H) * r;
  const unsigned short* W3 = W2 + int64_t(H) * H;
  for (int e = tid; e < R * H; e += NT) {
    const int b = e / H, j = e % H;
    float acc = p[o.b1 + j];
    for (int i = 0; i < r; ++i) acc += wb(W1, int64_t(j) * r + i) * x[b * r + i];
    if (z1) z1[e] = acc;
    a1[e] = bf16f(gelu_f(acc));
  }
  __syncthreads();
  for (int e = tid; e < R * H; e += NT) {
    const int b = e / H, j = e % H;
    float acc = p[o.b2 + j];
    for (int k = 0; k < H; ++k) acc += wb(W2, int64_t(j) * H + k) * a1[b * H + k];
    if (z2) z2[e] = acc;
    a2[e] = bf16f(gelu_f(acc));
  }
  __syncthreads();
  for (int e = tid; e < R * r; e += NT) {
    const int b = e / r, i = e % r;
    float acc = p[o.b3 + i];
    for (int j = 0; j < H; ++j) acc += wb(W3, int64_t(i) * H + j) * a2[b * H + j];
    out[e] = acc;
  }
  __syncthreads();
}

__device__ int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// visiting order of epoch e: i -> (a i + c) mod N, a advanced to be coprime with N
__device__ void epoch_coeffs(int64_t N, int64_t e, int64_t& a, int64_t& c) {
  if (N == 1) {
    a = 1;
    c = 0;
    return;
  }
  a = int64_t((uint64_t(e) * 2654435761ull + 1ull) % uint64_t(N));
  if (a == 0) a = 1;
  while (gcd64(a, N) != 1) a = (a + 1 < N) ? a + 1 : 1;
  c = int64_t((uint64_t(e) * 40503ull + 17ull) % uint64_t(N));
}

// ---- trainer and gradient on the matrix cores --------------------------------
// One workgroup of 8 waves runs a minibatch in chunks of CB = 32 rows.  Per
// chunk (all operands in LDS, r padded with zeros to RP = 32 or 64):
//   forward  z1 = x W1^T + b1, a1 = bf16(gelu(z1)); z2, a2 likewise;
//            out = a2 W3^T + b3               (v_mfma_f32_16x16x32_bf16:
//            bf16 x bf16 products are exact, sums in float32)
//   backward dout = 2 (out - y) / (R r); dz2 = (dout W3) * gelu'(z2);
//            dz1 = (dz2 W2) * gelu'(z1)      (v_mfma_f32_16x16x4f32)
//   weights  dW3 += dout^T a2, dW2 += dz2^T a1, dW1 += dz1^T x, bias sums
// gelu'(z) is kept instead of z and overwritten by dz in place.  The weight
// gradients stay in the accumulators of their owning lanes across chunks
// (wave w owns column block w of dW3 and dW2 and row block w of dW1), so the
// owner applies Adam to its entries and writes their new bfloat16 copies
// straight into the LDS weights of the next step.
constexpr int MT = 512;  // trainer threads
constexpr int CB = 32;   // rows per chunk
constexpr int BPAD = 8;  // bf16 row padding (16 bytes)
constexpr int FPAD = 4;  // fp32 row padding
constexpr int ADAM_W = 8;  // Adam entries per thread with their loads in flight together


template <int RP>
struct TL {  // LDS layout (byte offsets); pitches in elements
  static constexpr int LW1 = RP + BPAD, LW2 = H + BPAD, LW3 = H + BPAD;
  static constexpr int LX = RP + BPAD, LA = H + BPAD;
  static constexpr int LG = H + FPAD, LD = RP + FPAD, LY = RP;
  static constexpr size_t w1 = 0;
  static constexpr size_t w2 = w1 + size_t(H) * LW1 * 2;
  static constexpr size_t w3 = w2 + size_t(H) * LW2 * 2;
  static constexpr size_t bias = w3 + size_t(RP) * LW3 * 2;  // b1 (H) | b2 (H) | b3 (RP), float
  static constexpr size_t xs = bias + size_t(2 * H + RP) * 4;
  static constexpr size_t a1 = xs + size_t(CB) * LX * 2;
  static constexpr size_t a2 = a1 + size_t(CB) * LA * 2;
  static constexpr size_t g1 = a2 + size_t(CB) * LA * 2;
  static constexpr size_t g2 = g1 + size_t(CB) * LG * 4;
  static constexpr size_t dd = g2 + size_t(CB) * LG * 4;
  static constexpr size_t ys = dd + size_t(CB) * LD * 4;
  static constexpr size_t total = ys + size_t(CB) * LY * 4;
};

template <int RP>
struct TPtr {
  unsigned short *w1, *w2, *w3, *xs, *a1, *a2;
  float *bias, *g1, *g2, *dd, *ys;
  __device__ explicit TPtr(unsigned char* sm) {
    using L = TL<RP>;
    w1 = reinterpret_cast<unsigned short*>(sm + L::w1);
    w2 = reinterpret_cast<unsigned short*>(sm + L::w2);
    w3 = reinterpret_cast<unsigned short*>(sm + L::w3);
    bias = reinterpret_cast<float*>(sm + L::bias);
    xs = reinterpret_cast<unsigned short*>(sm + L::xs);
    a1 = reinterpret_cast<unsigned short*>(sm + L::a1);
    a2 = reinterpret_cast<unsigned short*>(sm + L::a2);
    g1 = reinterpret_cast<float*>(sm + L::g1);
    g2 = reinterpret_cast<float*>(sm + L::g2);
    dd = reinterpret_cast<float*>(sm + L::dd);
    ys = reinterpret_cast<float*>(sm + L::ys);
  }
};

// bfloat16 weights and float biases of params into LDS (padding zero);
// ld(index) reads one parameter
template <int RP, class Ld>
__device__ void load_weights(Ld ld, int r, const TPtr<RP>& t, int tid) {
  using L = TL<RP>;
  const Off o(r);
  for (int e = tid; e < H * L::LW1; e += MT) {
    const int j = e / L::LW1, i = e % L::LW1;
    t.w1[e] = (i < r) ? bf16_bits(ld(o.w1 + int64_t(j) * r + i)) : 0;
  }
  for (int e = tid; e < H * L::LW2; e += MT) {
    const int j = e / L::LW2, k = e % L::LW2;
    t.w2[e] = (k < H) ? bf16_bits(ld(o.w2 + int64_t(j) * H + k)) : 0;
  }
  for (int e = tid; e < RP * L::LW3; e += MT) {
    const int i = e / L::LW3, j = e % L::LW3;
    t.w3[e] = (i < r && j < H) ? bf16_bits(ld(o.w3 + int64_t(i) * H + j)) : 0;
  }
  for (int e = tid; e < 2 * H + RP; e += MT) {
    float b = 0.f;
    if (e < H)
      b = ld(o.b1 + e);
    else if (e < 2 * H)
      b = ld(o.b2 + e - H);
    else if (e - 2 * H < r)
      b = ld(o.b3 + e - 2 * H);
    t.bias[e] = b;
  }
}

// float stores that reach the level coherent between workgroups on different
// XCDs (relaxed device-scope atomics, as for the other persistent kernels)
__device__ __forceinline__ void st_coh(float* p, float v) {
  __hip_atomic_store(reinterpret_cast<unsigned*>(p), __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float bfv(const unsigned short* p, int i) { return __uint_as_float(unsigned(p[i]) << 16); }

// 16 x 16 block (rb, cb) of A W^T with A (rows) and W (rows = output columns)
// bfloat16 row-major in LDS, K a multiple of 32
template <int K>
__device__ __forceinline__ flt4 mm_bf16(const unsigned short* A, int lda, const unsigned short* W, int ldw, int rb,
                                        int cb, int lane) {
  flt4 acc = {0.f, 0.f, 0.f, 0.f};
  const unsigned short* ap = A + (rb * 16 + (lane & 15)) * lda + 8 * (lane >> 4);
  const unsigned short* wp = W + (cb * 16 + (lane & 15)) * ldw + 8 * (lane >> 4);
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 32) {
    const bf16x8 a = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(ap + k0));
    const bf16x8 b = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(wp + k0));
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// Per-step state of a lane: weight-gradient blocks and bias sums.
template <int RP>
struct GAcc {
  flt4 w3[RP / 16];  // dW3 (row block u, column block w)
  flt4 w2[8];        // dW2 (row block u, column block w)
  flt4 w1[RP / 16];  // dW1 (row block w, column block u)
  float db;          // tid < H: db1[tid]; H <= tid < 2H: db2; 2H <= tid < 2H + RP: db3
  float loss;        // this lane's share of sum (out - y)^2
};

// Rows [c_begin, c_end) of a minibatch of R rows (row b of the batch = data
// row rowof(b)), in chunks of CB: their share of the gradient of the
// minibatch's mean loss into g (zero when the range holds no rows).
template <int RP, class RowOf>
__device__ void batch_grad(int r, const double* __restrict__ X, const double* __restrict__ Y,
                           const double* __restrict__ norm, int R, int c_begin, int c_end, RowOf rowof,
                           const TPtr<RP>& t, GAcc<RP>& g) {
  using L = TL<RP>;
  const int tid = threadIdx.x, lane0 = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const float scale = 2.0f / float(R * r);
#pragma unroll
  for (int u = 0; u < RP / 16; ++u) g.w3[u] = g.w1[u] = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int u = 0; u < 8; ++u) g.w2[u] = flt4{0.f, 0.f, 0.f, 0.f};
  g.db = 0.f;
  g.loss = 0.f;
  const int fr = w & 1, fc = w >> 1;  // forward / dz block coordinates: rows fr, columns fc and fc + 4
  // this thread's entries of a chunk (element e = tid + MT q of CB x RP):
  // fetched into registers one chunk ahead, so their global loads fly while
  // the previous chunk is computed
  constexpr int NQ = CB * RP / MT;
  double xr[NQ], yr[NQ];
  auto fetch = [&](int c0) {
    const int Rc = min(CB, R - c0);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tid + MT * q, b = e / RP, i = e % RP;
      xr[q] = 0.0;
      yr[q] = 0.0;
      if (b < Rc && i < r) {
        const int64_t row = rowof(c0 + b);
        xr[q] = X[row * r + i];
        yr[q] = Y[row * r + i];
      }
    }
  };
  const int c_stop = min(R, c_end);
  if (c_begin < c_stop) fetch(c_begin);
  for (int c0 = c_begin; c0 < c_stop; c0 += CB) {
    const int Rc = min(CB, R - c0);
    // the lane index made opaque per chunk: keeps the compiler from hoisting
    // the chunk's many LDS addresses out of the batch and epoch loops, where
    // they would stay live (and spill) across the whole step
    int lane = lane0;
    asm volatile("" : "+v"(lane));
    // ---- chunk rows: standardized x (bf16) and y ---------------------------
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tid + MT * q, b = e / RP, i = e % RP;
      float xv = 0.f, yv = 0.f;
      if (b < Rc && i < r) {
        xv = bf16f(static_cast<float>((xr[q] - norm[i]) / norm[r + i]));
        yv = static_cast<float>((yr[q] - norm[2 * r + i]) / norm[3 * r + i]);
      }
      t.xs[b * L::LX + i] = bf16_bits(xv);
      t.ys[b * L::LY + i] = yv;
    }
    __syncthreads();
    if (c0 + CB < c_stop) fetch(c0 + CB);
    // ---- forward ------------------------------------------------------------
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int cb = fc + 4 * h;
      const flt4 acc = mm_bf16<RP>(t.xs, L::LX, t.w1, L::LW1, fr, cb, lane);
      const int col = cb * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = fr * 16 + 4 * (lane >> 4) + e;
        const float z = acc[e] + t.bias[col];
        t.a1[row * L::LA + col] = bf16_bits(gelu_f(z));
        t.g1[row * L::LG + col] = gelu_grad_f(z);
      }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int cb = fc + 4 * h;
      const flt4 acc = mm_bf16<H>(t.a1, L::LA, t.w2, L::LW2, fr, cb, lane);
      const int col = cb * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = fr * 16 + 4 * (lane >> 4) + e;
        const float z = acc[e] + t.bias[H + col];
        t.a2[row * L::LA + col] = bf16_bits(gelu_f(z));
        t.g2[row * L::LG + col] = gelu_grad_f(z);
      }
    }
    __syncthreads();
    if (w < 2 * (RP / 16)) {  // out and dout, blocks (w & 1, w >> 1)
      const flt4 acc = mm_bf16<H>(t.a2, L::LA, t.w3, L::LW3, fr, fc, lane);
      const int col = fc * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = fr * 16 + 4 * (lane >> 4) + e;
        float d = 0.f;
        if (row < Rc && col < r) d = (acc[e] + t.bias[2 * H + col]) - t.ys[row * L::LY + col];
        g.loss += d * d;
        t.dd[row * L::LD + col] = scale * d;
      }
    }
    __syncthreads();
    // ---- dz2 = (dout W3) * gelu'(z2) in place; dW3 += dout^T a2 -------------
    {  // blocks (fr, fc) and (fr, fc + 4) share their A fragments
      flt4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll 4
      for (int k0 = 0; k0 < RP; k0 += 4) {
        const int k = k0 + (lane >> 4);
        const float av = t.dd[(fr * 16 + (lane & 15)) * L::LD + k];
#pragma unroll
        for (int h = 0; h < 2; ++h)
          acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bfv(t.w3, k * L::LW3 + (fc + 4 * h) * 16 + (lane & 15)),
                                                        acc[h], 0, 0, 0);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int col = (fc + 4 * h) * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = fr * 16 + 4 * (lane >> 4) + e;
          t.g2[row * L::LG + col] *= acc[h][e];
        }
      }
    }
#pragma unroll 2
    for (int k0 = 0; k0 < CB; k0 += 4) {
      const int b = k0 + (lane >> 4);
      const float bv = bfv(t.a2, b * L::LA + w * 16 + (lane & 15));
#pragma unroll
      for (int u = 0; u < RP / 16; ++u)
        g.w3[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(t.dd[b * L::LD + u * 16 + (lane & 15)], bv, g.w3[u], 0, 0, 0);
    }
    __syncthreads();
    // ---- dz1 = (dz2 W2) * gelu'(z1) in place; dW2 += dz2^T a1 ----------------
    {
      flt4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll 4
      for (int k0 = 0; k0 < H; k0 += 4) {
        const int k = k0 + (lane >> 4);
        const float av = t.g2[(fr * 16 + (lane & 15)) * L::LG + k];
#pragma unroll
        for (int h = 0; h < 2; ++h)
          acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bfv(t.w2, k * L::LW2 + (fc + 4 * h) * 16 + (lane & 15)),
                                                        acc[h], 0, 0, 0);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int col = (fc + 4 * h) * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = fr * 16 + 4 * (lane >> 4) + e;
          t.g1[row * L::LG + col] *= acc[h][e];
        }
      }
    }
#pragma unroll 2
    for (int k0 = 0; k0 < CB; k0 += 4) {
      const int b = k0 + (lane >> 4);
      const float bv = bfv(t.a1, b * L::LA + w * 16 + (lane & 15));
#pragma unroll
      for (int u = 0; u < 8; ++u)
        g.w2[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(t.g2[b * L::LG + u * 16 + (lane & 15)], bv, g.w2[u], 0, 0, 0);
    }
    __syncthreads();
    // ---- dW1 += dz1^T x; bias sums --------------------------------------------
#pragma unroll 2
    for (int k0 = 0; k0 < CB; k0 += 4) {
      const int b = k0 + (lane >> 4);
      const float av = t.g1[b * L::LG + w * 16 + (lane & 15)];
#pragma unroll
      for (int u = 0; u < RP / 16; ++u)
        g.w1[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bfv(t.xs, b * L::LX + u * 16 + (lane & 15)), g.w1[u], 0, 0, 0);
    }
    // bias sums over all CB rows (rows past the batch hold zero gradients),
    // every load in flight before the adds: threads 0..127 db1, 128..255
    // db2, 256..256+RP-1 db3
    if (tid < 2 * H + RP) {
      const float* src = tid < H ? t.g1 + tid : (tid < 2 * H ? t.g2 + (tid - H) : t.dd + (tid - 2 * H));
      const int pitch = tid < 2 * H ? L::LG : L::LD;
      float va[CB];
#pragma unroll
      for (int b = 0; b < CB; ++b) va[b] = src[b * pitch];
      float sa = 0.f;
#pragma unroll
      for (int b = 0; b < CB; ++b) sa += va[b];
      g.db += sa;
    }
    __syncthreads();
  }
}

// Visit every gradient entry this lane owns: f(parameter index, gradient).
template <int RP, class F>
__device__ void for_owned(int r, const TPtr<RP>& t, const GAcc<RP>& g, F f) {
  const Off o(r);
  const int tid = threadIdx.x, w = tid >> 6;
  int lane = tid & 63;
  asm volatile("" : "+v"(lane));  // no index hoisted out of the caller's loops
#pragma unroll
  for (int u = 0; u < RP / 16; ++u)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = u * 16 + 4 * (lane >> 4) + e, j = w * 16 + (lane & 15);  // dW3[i][j]
      if (i < r) f(o.w3 + int64_t(i) * H + j, g.w3[u][e]);
      const int j1 = w * 16 + 4 * (lane >> 4) + e, i1 = u * 16 + (lane & 15);  // dW1[j1][i1]
      if (i1 < r) f(o.w1 + int64_t(j1) * r + i1, g.w1[u][e]);
    }
#pragma unroll
  for (int u = 0; u < 8; ++u)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = u * 16 + 4 * (lane >> 4) + e, k = w * 16 + (lane & 15);  // dW2[j][k]
      f(o.w2 + int64_t(j) * H + k, g.w2[u][e]);
    }
  if (tid < H)
    f(o.b1 + tid, g.db);
  else if (tid < 2 * H)
    f(o.b2 + tid - H, g.db);
  else if (tid < 2 * H + r)
    f(o.b3 + tid - 2 * H, g.db);
  (void)t;
}

// Float image of the LDS weights: the bfloat16 arrays w1 | w2 | w3 (with
// their padding, same order) as floats, then b1 | b2 | b3.  The Adam step
// writes each parameter's new value at its place; every workgroup then
// converts the whole image into its LDS with 16-byte loads.
template <int RP>
struct Img {
  using L = TL<RP>;
  static constexpr int NWB = H * L::LW1 + H * L::LW2 + RP * L::LW3;  // weight entries
  static constexpr int N = NWB + 2 * H + RP;
};

// image position of parameter e
template <int RP>
__device__ int img_index(int r, int e) {
  using L = TL<RP>;
  const int b1 = H * r, w2 = b1 + H, b2 = w2 + H * H, w3 = b2 + H, b3 = w3 + r * H;
  constexpr int o2 = H * L::LW1, o3 = o2 + H * L::LW2, ob = Img<RP>::NWB;
  if (e < b1) {
    const int j = e / r;
    return j * L::LW1 + (e - j * r);
  }
  if (e < w2) return ob + (e - b1);
  if (e < b2) return o2 + ((e - w2) / H) * L::LW2 + (e - w2) % H;
  if (e < w3) return ob + H + (e - b2);
  if (e < b3) return o3 + ((e - w3) / H) * L::LW3 + (e - w3) % H;
  return ob + 2 * H + (e - b3);
}

// the image into the LDS weights and biases (all of a thread's loads in
// flight); the caller has invalidated its caches (acquire fence) after the
// other workgroups' device-coherent stores
template <int RP>
__device__ void reload_weights(const float* img, const TPtr<RP>& t, int tid) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  typedef unsigned short u4 __attribute__((ext_vector_type(4)));
  constexpr int Q = Img<RP>::N / 4, QW = Img<RP>::NWB / 4;
  constexpr int RW = 9;  // loads per thread in flight; two passes cover r <= 64
  for (int q0 = tid; q0 < Q; q0 += RW * MT) {
    f4 v[RW];
#pragma unroll
    for (int u = 0; u < RW; ++u) {
      const int q = q0 + u * MT;
      v[u] = (q < Q) ? reinterpret_cast<const f4*>(img)[q] : f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < RW; ++u) {
      const int q = q0 + u * MT;
      if (q < QW) {
        u4 b;
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = bf16_bits(v[u][c]);
        *reinterpret_cast<u4*>(t.w1 + 4 * q) = b;  // w1 | w2 | w3 are contiguous
      } else if (q < Q) {
        *reinterpret_cast<f4*>(t.bias + 4 * (q - QW)) = v[u];
      }
    }
  }
}

// workgroup sum of the lanes' loss shares (every thread gets it)
__device__ float block_loss(float v, float* red) {
  v = float(wave_sum(double(v)));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float s = 0.f;
  for (int i = 0; i < MT / 64; ++i) s += red[i];
  return s;
}

struct TrainArgs {
  int r;
  const double* X;
  const double* Y;
  int64_t N;
  int epochs, batch;
  float lr, beta1, beta2, eps;
  float* params;
  const double* norm;
  float* m;
  float* v;
  float* Gpart;     // per workgroup: its share of the minibatch gradient (P floats each)
  float* lpart;     // per workgroup: its share of the minibatch's squared error
  float* img;       // float image of the LDS weights (Img)
  unsigned* words;  // [0] barrier counter, [1] abort flag (zero at launch)
  float* loss_log;
};

// One cooperative launch of ceil(batch / CB) workgroups runs every epoch.
// Per minibatch, workgroup w takes rows [CB w, CB w + CB): forward, backward
// and its share of the gradient (batch_grad), stored to Gpart[w]; a
// device-wide barrier; then each workgroup sums the shares of its slice of
// the P parameters in workgroup order (deterministic) and applies Adam to
// that slice (m and v stay with their workgroup); a second barrier; then
// every workgroup reads the new parameters into its LDS weights.  Shared
// data is stored with device-coherent stores and read with plain loads
// after an acquire fence that invalidates the reader's caches.  A barrier that times
// out raises the abort flag: every workgroup leaves and the loss log reads
// NaN from that epoch on.
template <int RP>
__global__ __launch_bounds__(MT) void train_kernel(TrainArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ float red[MT / 64];
  __shared__ int rows_sh[BMAX];  // the minibatch's data rows
  const int tid = threadIdx.x;
  const int wg = blockIdx.x, nw = gridDim.x;
  const int r = a.r;
  const Off o(r);
  const TPtr<RP> t(smem);
  const int P = int(o.P);
  const int lo = int(int64_t(P) * wg / nw), hi = int(int64_t(P) * (wg + 1) / nw);  // this workgroup's Adam slice
  float* __restrict__ mp = a.m;
  float* __restrict__ vp = a.v;
  for (int e = lo + tid; e < hi; e += MT) {
    mp[e] = 0.f;
    vp[e] = 0.f;
  }
  load_weights<RP>([&](int64_t e) { return a.params[e]; }, r, t, tid);
  __syncthreads();
  if (wg == 0) {  // the image of the initial weights, padding included
    const unsigned short* wb = t.w1;
    for (int q = tid; q < Img<RP>::NWB; q += MT) st_coh(a.img + q, bfv(wb, q));
    for (int q = tid; q < 2 * H + RP; q += MT) st_coh(a.img + Img<RP>::NWB + q, t.bias[q]);
  }
  unsigned gen = 0;
  unsigned* bar = a.words;
  int* abort_flag = reinterpret_cast<int*>(a.words + 1);
  GAcc<RP> g;
  int64_t step = 0;
  for (int ep = 0; ep < a.epochs; ++ep) {
    int64_t ca, cc;
    epoch_coeffs(a.N, ep, ca, cc);
    double ltot = 0.0;
    bool ok = true;
    for (int64_t s0 = 0; s0 < a.N && ok; s0 += a.batch) {
      const int R = int(min<int64_t>(a.batch, a.N - s0));
      for (int b = tid; b < R; b += MT) rows_sh[b] = int((ca * (s0 + b) + cc) % a.N);
      __syncthreads();
      batch_grad<RP>(r, a.X, a.Y, a.norm, R, wg * CB, wg * CB + CB, [&](int b) { return int64_t(rows_sh[b]); }, t,
                     g);
      const float lsum = block_loss(g.loss, red);
      float* gmine = a.Gpart + int64_t(wg) * P;
      for_owned<RP>(r, t, g, [&](int64_t e, float gr) { st_coh(gmine + e, gr); });
      if (tid == 0) st_coh(a.lpart + wg, lsum);
      if (!xwg::team_barrier(bar, unsigned(nw), gen, abort_flag)) {
        ok = false;
        break;
      }
      // drop this CU's and this XCD's cached copies of data that other
      // workgroups stored (their stores went to the coherent level), so
      // plain loads, which the compiler may batch, read the new values
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      float ls = 0.f;
      for (int q = 0; q < nw; ++q) ls += a.lpart[q];
      ltot += double(ls / float(R * r)) * R;
      ++step;
      // Adam (Kingma & Ba 2015; bias corrections in double) on this
      // workgroup's slice, ADAM_W entries per thread with their loads in flight
      const float c1 = static_cast<float>(1.0 - pow(double(a.beta1), double(step)));
      const float c2 = static_cast<float>(1.0 - pow(double(a.beta2), double(step)));
      for (int e0 = lo + tid; e0 < hi; e0 += ADAM_W * MT) {
        float gr[ADAM_W], mo[ADAM_W], vo[ADAM_W], po[ADAM_W];
#pragma unroll
        for (int u = 0; u < ADAM_W; ++u) {
          const int e = e0 + u * MT;
          gr[u] = mo[u] = vo[u] = po[u] = 0.f;
          if (e < hi) {
            float sh[BMAX / CB];  // the shares, all loads in flight, summed in order
#pragma unroll
            for (int q = 0; q < BMAX / CB; ++q) sh[q] = (q < nw) ? a.Gpart[int64_t(q) * P + e] : 0.f;
#pragma unroll
            for (int q = 0; q < BMAX / CB; ++q) gr[u] += sh[q];
            mo[u] = mp[e];
            vo[u] = vp[e];
            po[u] = a.params[e];
          }
        }
#pragma unroll
        for (int u = 0; u < ADAM_W; ++u) {
          const int e = e0 + u * MT;
          if (e < hi) {
            const float mm = a.beta1 * mo[u] + (1.0f - a.beta1) * gr[u];
            const float vv = a.beta2 * vo[u] + (1.0f - a.beta2) * gr[u] * gr[u];
            mp[e] = mm;
            vp[e] = vv;
            const float pn = po[u] - a.lr * (mm / c1) / (sqrtf(vv / c2) + a.eps);
            st_coh(a.params + e, pn);
            st_coh(a.img + img_index<RP>(r, e), pn);
          }
        }
      }
      if (!xwg::team_barrier(bar, unsigned(nw), gen, abort_flag)) {
        ok = false;
        break;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      reload_weights<RP>(a.img, t, tid);
      __syncthreads();
    }
    if (!ok) {
      if (wg == 0 && tid == 0 && a.loss_log)
        for (int e = ep; e < a.epochs; ++e) a.loss_log[e] = __builtin_nanf("");
      return;
    }
    if (wg == 0 && tid == 0 && a.loss_log) a.loss_log[ep] = static_cast<float>(ltot / double(a.N));
  }
}

struct GradArgs {
  int r;
  const double* X;
  const double* Y;
  int64_t N;
  const float* params;
  const double* norm;
  float* G;
  float* loss;
};

// gradient of the mean loss over N <= BMAX rows
template <int RP>
__global__ __launch_bounds__(MT) void grad_kernel(GradArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ float red[MT / 64];
  const int tid = threadIdx.x;
  const TPtr<RP> t(smem);
  load_weights<RP>([&](int64_t e) { return a.params[e]; }, a.r, t, tid);
  __syncthreads();
  GAcc<RP> g;
  const int R = int(a.N);
  batch_grad<RP>(a.r, a.X, a.Y, a.norm, R, 0, R, [](int b) { return int64_t(b); }, t, g);
  const float loss = block_loss(g.loss, red) / float(R * a.r);
  for_owned<RP>(a.r, t, g, [&](int64_t e, float gr) { a.G[e] = gr; });
  if (tid == 0) *a.loss = loss;
}

__global__ void zero_u32_kernel(unsigned* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// per-mode statistics of X and Y (N x r each): norm = [mx | sx | my | sy]
__global__ void norm_kernel(const double* __restrict__ X, const double* __restrict__ Y, int64_t N, int r,
                            double* __restrict__ norm) {
  __shared__ double red[4];
  const int i = blockIdx.x % r;
  const bool isy = blockIdx.x >= r;
  const double* A = isy ? Y : X;
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < N; t += 256) s += A[t * r + i];
  s = block_sum<256>(s, red);
  const double m = s / double(N);
  double q = 0.0;
  for (int64_t t = threadIdx.x; t < N; t += 256) {
    const double d = A[t * r + i] - m;
    q += d * d;
  }
  q = block_sum<256>(q, red);
  double sd = sqrt(q / double(N));
  if (!(sd > 0.0)) sd = 1.0;
  if (threadIdx.x == 0) {
    norm[(isy ? 2 : 0) * r + i] = m;
    norm[(isy ? 3 : 1) * r + i] = sd;
  }
}

// rho_t = qhat_{t+1} - f_ROM(qhat_t): one workgroup per t
__global__ __launch_bounds__(256) void residual_kernel(const double* __restrict__ O, int r,
                                                       const double* __restrict__ Qhat, int64_t ldqh, int64_t k,
                                                       double* __restrict__ R) {
  extern __shared__ double fsh[];
  const int64_t t = blockIdx.x;
  const int64_t s = nquad(r), d = ncols(r);
  for (int64_t c = threadIdx.x; c < d; c += 256) {
    double v;
    if (c < r) {
      v = Qhat[c * ldqh + t];
    } else if (c < r + s) {
      int ii = 0;
      int64_t off = 0, q = c - r;
      while (off + (r - ii) <= q) {
        off += r - ii;
        ++ii;
      }
      const int jj = ii + int(q - off);
      v = Qhat[int64_t(ii) * ldqh + t] * Qhat[int64_t(jj) * ldqh + t];
    } else {
      v = 1.0;
    }
    fsh[c] = v;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = w; i < r; i += 4) {
    double acc = 0.0;
    for (int64_t c = lane; c < d; c += 64) acc += O[int64_t(i) * d + c] * fsh[c];
    acc = wave_sum(acc);
    if (lane == 0) R[t * r + i] = Qhat[int64_t(i) * ldqh + t + 1] - acc;
  }
}

// g(x) for RG rows per workgroup, physical units; gnorm[row] = ||g(x_row)||
__global__ __launch_bounds__(ET) void eval_kernel(int r, const float* __restrict__ p, const double* __restrict__ norm,
                                                  const double* __restrict__ X, int64_t N, double* __restrict__ Gout,
                                                  double* __restrict__ gnorm) {
  extern __shared__ unsigned char smem[];
  const Off o(r);
  unsigned short* Wb = reinterpret_cast<unsigned short*>(smem);
  float* x = reinterpret_cast<float*>(smem + round_up(size_t(o.P - 2 * H - r) * 2, 16));
  float* a1 = x + RG * r;
  float* a2 = a1 + RG * H;
  float* out = a2 + RG * H;
  const int tid = threadIdx.x;
  const int64_t row0 = int64_t(blockIdx.x) * RG;
  const int R = int(min<int64_t>(RG, N - row0));
  load_wb(p, r, Wb, tid, ET);
  for (int e = tid; e < RG * r; e += ET) {
    const int b = e / r, i = e % r;
    x[e] = (b < R) ? bf16f(static_cast<float>((X[(row0 + b) * r + i] - norm[i]) / norm[r + i])) : 0.f;
  }
  __syncthreads();
  mlp_fwd<ET>(RG, r, Wb, p, x, nullptr, a1, nullptr, a2, out, tid);
  for (int b = tid / 64; b < R; b += ET / 64) {
    double n2 = 0.0;
    for (int i = tid % 64; i < r; i += 64) {
      const double g = double(out[b * r + i]) * norm[3 * r + i] + norm[2 * r + i];
      if (Gout) Gout[(row0 + b) * r + i] = g;
      n2 += g * g;
    }
    n2 = wave_sum(n2);
    if (tid % 64 == 0) gnorm[row0 + b] = sqrt(n2);
  }
}

__global__ void max_kernel(const double* __restrict__ v, int64_t n, double* __restrict__ out) {
  __shared__ double red[4];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, v[i]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) *out = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

struct CRollArgs {
  int r;
  const double* O;
  const float* p;
  const double* norm;
  double threshold;  // <= 0: closure off
  const double* q0;  // M x r
  int64_t M;
  int n_states;
  const double* Qref;  // r x k_ref (ld ldref): error reference and growth statistics
  int64_t ldref, k_ref;
  const double* mean;  // r, temporal mean of Qref
  const double* maxdev;
  double max_growth;
  double* traj;  // M x n_states x r or null
  double* err;
  double* growth;
  int* outcome;
  int* fallback_at;
};

// ---- closure rollouts ------------------------------------------------------
// CR (4, or 2 when the operator streams) states per workgroup of CT threads
// (8 waves).  The MLP runs on the matrix
// cores (v_mfma_f32_16x16x32_bf16, the CR states padded to 16 rows): the bf16
// weights sit in LDS row-major with rows padded by 8 elements so that the 16
// lanes reading one operand column hit 16 different bank groups; activations
// are rounded to bf16 exactly where the trainer rounds them.  The features
// [q | quad(q) | 1 | 0...] of the CR states sit in LDS; wave w owns ROM rows
// w, w+8, ..., and, when RES is set (r <= 40, d <= 1024), keeps them in
// registers for the whole rollout, so the operator is read once; otherwise
// its rows stream from L2, coalesced.
constexpr int CR_RES = 4;      // states per workgroup when the operator is resident (r <= 40)
constexpr int CR_STREAM = 2;   // states per workgroup otherwise (LDS holds their features)
constexpr int CT = 512;        // threads per workgroup
constexpr int CW = CT / 64;    // waves
constexpr int RES_ROWS = 5;    // rows per wave kept in registers (r <= 40)
constexpr int RES_NJ = 16;     // columns per lane kept in registers (d <= 1024)
constexpr int MPAD = 8;        // bf16 padding per LDS row of an MFMA operand

struct RollLds {  // byte offsets into the rollout kernel's LDS
  int r, rp, rp16, p1, p2;    // K of layer 1 padded to 32, N of layer 3 padded to 16, row pitches
  int64_t dpad;
  size_t w1, w2, w3, xa, a1a, a2a, F, q, qn, mean, stat, gout, flag, qi, total;
  __host__ __device__ RollLds(int rr, int CR) {
    r = rr;
    rp = int(round_up(size_t(r), 32));
    rp16 = int(round_up(size_t(r), 16));
    p1 = rp + MPAD;
    p2 = H + MPAD;
    dpad = int64_t(round_up(size_t(ncols(r)), 64));
    size_t o = 0;
    w1 = o; o += round_up(size_t(H) * p1 * 2, 16);        // W1 [H][p1]
    w2 = o; o += round_up(size_t(H) * p2 * 2, 16);        // W2 [H][p2]
    w3 = o; o += round_up(size_t(rp16) * p2 * 2, 16);     // W3 [rp16][p2]
    xa = o; o += round_up(size_t(16) * p1 * 2, 16);       // x  [16][p1]
    a1a = o; o += round_up(size_t(16) * p2 * 2, 16);      // a1 [16][p2]
    a2a = o; o += round_up(size_t(16) * p2 * 2, 16);      // a2 [16][p2]
    F = o; o += size_t(CR) * dpad * 8;
    q = o; o += size_t(CR) * r * 8;
    qn = o; o += size_t(CR) * r * 8;
    mean = o; o += size_t(r) * 8;
    stat = o; o += size_t(CR) * 2 * 8;
    gout = o; o += round_up(size_t(CR) * r * 4, 16);
    flag = o; o += size_t(CR) * 2 * 4;
    qi = o; o += size_t(2) * nquad(r) * 2;
    total = round_up(o, 16) + 64;
  }
};

// One 16x16 output block of a 16-row layer: C = A (16 x K) . W^T, with W
// row-major [N][pitch] and A row-major [16][pitch], K a multiple of 32.
__device__ __forceinline__ flt4 mlp_block(const unsigned short* A, int pa, const unsigned short* W, int pw, int n0,
                                          int K, int lane) {
  flt4 c = {0.f, 0.f, 0.f, 0.f};
  const int m = lane & 15, kq = (lane >> 4) * 8;
  for (int k0 = 0; k0 < K; k0 += 32) {
    const bf16x8 av = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(A + m * pa + k0 + kq));
    const bf16x8 bv = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(W + (n0 + m) * pw + k0 + kq));
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  }
  return c;  // lane l, element e: row 4 (l / 16) + e, column n0 + l % 16
}

template <bool RES>
__global__ __launch_bounds__(CT) void closure_rollout_kernel(CRollArgs a) {
  constexpr int CR = RES ? CR_RES : CR_STREAM;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int r = a.r;
  const Off o(r);
  const RollLds L(r, CR);
  const int64_t s = nquad(r), d = ncols(r);
  const int64_t dpad = L.dpad;
  const int NJ = int(dpad / 64);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  unsigned short* W1 = reinterpret_cast<unsigned short*>(smem + L.w1);
  unsigned short* W2 = reinterpret_cast<unsigned short*>(smem + L.w2);
  unsigned short* W3 = reinterpret_cast<unsigned short*>(smem + L.w3);
  unsigned short* XA = reinterpret_cast<unsigned short*>(smem + L.xa);
  unsigned short* A1 = reinterpret_cast<unsigned short*>(smem + L.a1a);
  unsigned short* A2 = reinterpret_cast<unsigned short*>(smem + L.a2a);
  double* F = reinterpret_cast<double*>(smem + L.F);
  double* q = reinterpret_cast<double*>(smem + L.q);
  double* qn = reinterpret_cast<double*>(smem + L.qn);
  double* mean = reinterpret_cast<double*>(smem + L.mean);
  double* stat = reinterpret_cast<double*>(smem + L.stat);  // per state: err2max, devmax
  float* gout = reinterpret_cast<float*>(smem + L.gout);
  int* flag = reinterpret_cast<int*>(smem + L.flag);         // per state: latched step (-1), non-finite (0/1)
  unsigned short* qi = reinterpret_cast<unsigned short*>(smem + L.qi);
  unsigned short* qj = qi + s;

  const int64_t m0 = int64_t(blockIdx.x) * CR;
  const int R = int(min<int64_t>(CR, a.M - m0));
  const bool use_g = a.threshold > 0.0;
  // zero everything the MLP reads (padding rows and columns stay zero), then the weights
  for (size_t e = tid; e < (L.F - L.w1) / 2; e += CT) W1[e] = 0;
  __syncthreads();
  if (use_g) {
    for (int64_t e = tid; e < int64_t(H) * r; e += CT) W1[(e / r) * L.p1 + e % r] = bf16_bits(a.p[o.w1 + e]);
    for (int64_t e = tid; e < int64_t(H) * H; e += CT) W2[(e / H) * L.p2 + e % H] = bf16_bits(a.p[o.w2 + e]);
    for (int64_t e = tid; e < int64_t(r) * H; e += CT) W3[(e / H) * L.p2 + e % H] = bf16_bits(a.p[o.w3 + e]);
  }
  for (int64_t c = tid; c < s; c += CT) {
    int ii = 0;
    int64_t off = 0;
    while (off + (r - ii) <= c) {
      off += r - ii;
      ++ii;
    }
    qi[c] = static_cast<unsigned short>(ii);
    qj[c] = static_cast<unsigned short>(ii + (c - off));
  }
  for (int64_t e = tid; e < int64_t(CR) * dpad; e += CT) F[e] = 0.0;
  for (int e = tid; e < CR * r; e += CT) q[e] = (e / r < R) ? a.q0[(m0 + e / r) * r + e % r] : 0.0;
  for (int i = tid; i < r; i += CT) mean[i] = a.mean[i];
  for (int b = tid; b < CR; b += CT) {
    stat[b * 2 + 0] = 0.0;
    stat[b * 2 + 1] = 0.0;
    flag[b * 2 + 0] = -1;
    flag[b * 2 + 1] = 0;
  }
  // resident operator rows: wave w owns rows w + 8u
  double orow[RES ? RES_ROWS : 1][RES ? RES_NJ : 1];
  if constexpr (RES) {
#pragma unroll
    for (int u = 0; u < RES_ROWS; ++u)
#pragma unroll
      for (int j = 0; j < RES_NJ; ++j) {
        const int i = w + CW * u;
        const int64_t c = lane + 64 * j;
        orow[u][j] = (i < r && c < d) ? a.O[int64_t(i) * d + c] : 0.0;
      }
  }
  __syncthreads();
  double maxdev = 0.0;
  for (int i = 0; i < r; ++i) maxdev = fmax(maxdev, a.maxdev[i]);

  // reference snapshot of the state being scored (lane i < r), one step ahead
  double href = (lane < r && 0 < a.k_ref) ? a.Qref[int64_t(lane) * a.ldref] : 0.0;
  for (int t = 0; t < a.n_states; ++t) {
    // ---- score state t: one wave per state (r <= 64: one mode per lane) ----
    if (w < R) {
      const int b = w;
      double e2 = 0.0, n2 = 0.0, dv = 0.0, bad = 0.0;
      if (lane < r) {
        const double xv = q[b * r + lane];
        if (!isfinite(xv)) bad = 1.0;
        dv = fabs(xv - mean[lane]);
        if (t < a.k_ref) {
          e2 = (xv - href) * (xv - href);
          n2 = href * href;
        }
        if (a.traj) a.traj[((m0 + b) * a.n_states + t) * r + lane] = xv;
      }
      e2 = wave_sum_dpp(e2);
      n2 = wave_sum_dpp(n2);
      dv = wave_max_dpp(dv);
      bad = wave_max_dpp(bad);
      if (lane == 0) {
        if (bad != 0.0) flag[b * 2 + 1] = 1;
        stat[b * 2 + 1] = fmax(stat[b * 2 + 1], dv);
        if (t < a.k_ref) stat[b * 2 + 0] = fmax(stat[b * 2 + 0], e2 / n2);
      }
    }
    if (t + 1 == a.n_states) break;
    href = (lane < r && t + 1 < a.k_ref) ? a.Qref[int64_t(lane) * a.ldref + t + 1] : 0.0;
    // ---- features of the CR states ----
    for (int e = tid; e < CR * r; e += CT) F[(e / r) * dpad + e % r] = q[e];
    for (int64_t e = tid; e < int64_t(CR) * s; e += CT) {
      const int b = int(e / s);
      const int64_t c = e % s;
      F[b * dpad + r + c] = q[b * r + qi[c]] * q[b * r + qj[c]];
    }
    if (tid < CR) F[tid * dpad + d - 1] = 1.0;
    // ---- closure g(q_t) on the matrix cores ----
    if (use_g) {
      for (int e = tid; e < CR * r; e += CT) {
        const int b = e / r, i = e % r;
        const double xv = q[e];
        XA[b * L.p1 + i] =
            bf16_bits(static_cast<float>((isfinite(xv) ? xv : 0.0) - a.norm[i]) / static_cast<float>(a.norm[r + i]));
      }
      __syncthreads();
      {  // layer 1: wave w -> hidden units 16w .. 16w+15
        const flt4 c = mlp_block(XA, L.p1, W1, L.p1, 16 * w, L.rp, lane);
        if (lane < 16)
#pragma unroll
          for (int e = 0; e < CR; ++e) A1[e * L.p2 + 16 * w + lane] = bf16_bits(gelu_f(c[e] + a.p[o.b1 + 16 * w + lane]));
      }
      __syncthreads();
      {  // layer 2
        const flt4 c = mlp_block(A1, L.p2, W2, L.p2, 16 * w, H, lane);
        if (lane < 16)
#pragma unroll
          for (int e = 0; e < CR; ++e) A2[e * L.p2 + 16 * w + lane] = bf16_bits(gelu_f(c[e] + a.p[o.b2 + 16 * w + lane]));
      }
      __syncthreads();
      if (16 * w < r) {  // layer 3: wave w -> outputs 16w .. 16w+15
        const flt4 c = mlp_block(A2, L.p2, W3, L.p2, 16 * w, H, lane);
        const int i = 16 * w + lane;
        if (lane < 16 && i < r)
#pragma unroll
          for (int e = 0; e < CR; ++e) gout[e * r + i] = c[e] + a.p[o.b3 + i];
      }
      __syncthreads();
      if (w < R) {
        const int b = w;
        double n2 = 0.0;
        if (lane < r) {
          const double g = double(gout[b * r + lane]) * a.norm[3 * r + lane] + a.norm[2 * r + lane];
          n2 = g * g;
        }
        n2 = wave_sum_dpp(n2);
        if (lane == 0 && flag[b * 2] < 0 && !(sqrt(n2) <= a.threshold)) flag[b * 2] = t;  // latch
      }
    }
    __syncthreads();
    // ---- ROM step: qn[b][i] = O[i, :] . F[b] (+ g) ----
    auto finish = [&](double acc, int b, int i) {
      acc = wave_sum_dpp(acc);
      if (lane == 0) {
        if (use_g && flag[b * 2] < 0) acc += double(gout[b * r + i]) * a.norm[3 * r + i] + a.norm[2 * r + i];
        qn[b * r + i] = acc;
      }
    };
    if constexpr (RES) {
      // fully unrolled so the resident rows stay in registers; each feature
      // value is read once and feeds the wave's rows
#pragma unroll
      for (int b = 0; b < CR; ++b) {
        double acc[RES_ROWS];
#pragma unroll
        for (int u = 0; u < RES_ROWS; ++u) acc[u] = 0.0;
#pragma unroll
        for (int j = 0; j < RES_NJ; ++j)
          if (j < NJ) {  // stay inside row b of F
            const double fv = F[b * dpad + lane + 64 * j];
#pragma unroll
            for (int u = 0; u < RES_ROWS; ++u) acc[u] += orow[u][j] * fv;
          }
#pragma unroll
        for (int u = 0; u < RES_ROWS; ++u)
          if (w + CW * u < r) finish(acc[u], b, w + CW * u);  // wave-uniform
      }
    } else {
      for (int u = 0; u < (r + CW - 1) / CW; ++u) {
        const int i = w + CW * u;
        if (i >= r) break;  // wave-uniform
#pragma unroll
        for (int b = 0; b < CR; ++b) {
          double acc = 0.0;
          for (int j = 0; j < NJ; ++j) {
            const int64_t c = lane + 64 * j;
            if (c < d) acc += a.O[int64_t(i) * d + c] * F[b * dpad + c];
          }
          finish(acc, b, i);
        }
      }
    }
    __syncthreads();
    for (int e = tid; e < CR * r; e += CT) q[e] = qn[e];
    __syncthreads();
  }
  for (int b = tid; b < R; b += CT) {
    const int64_t m = m0 + b;
    const bool nonfinite = flag[b * 2 + 1] != 0;
    const double gr = stat[b * 2 + 1] / maxdev;
    a.err[m] = nonfinite ? NAN : sqrt(stat[b * 2 + 0]);
    a.growth[m] = nonfinite ? NAN : gr;
    a.outcome[m] = nonfinite ? DOPINF_ITEM_NONFINITE : (gr < a.max_growth ? DOPINF_ITEM_PASS : DOPINF_ITEM_GROWTH);
    a.fallback_at[m] = flag[b * 2];
  }
}

__global__ __launch_bounds__(256) void ref_stats_kernel(const double* __restrict__ Q, int64_t ld, int64_t k,
                                                        double* __restrict__ mean, double* __restrict__ maxdev) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  const double* q = Q + int64_t(i) * ld;
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < k; t += 256) s += q[t];
  s = block_sum<256>(s, red);
  const double m = s / double(k);
  double mx = 0.0;
  for (int64_t t = threadIdx.x; t < k; t += 256) mx = fmax(mx, fabs(q[t] - m));
  mx = wave_max(mx);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    mean[i] = m;
    maxdev[i] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  }
}

size_t wb_bytes(int r) { return round_up(size_t(Off(r).P - 2 * H - r) * 2, 16); }
size_t train_lds(int r) { return r <= 32 ? TL<32>::total : TL<64>::total; }
size_t eval_lds(int r) { return wb_bytes(r) + round_up(size_t(RG) * r * 4, 16) + size_t(RG) * 2 * H * 4 + round_up(size_t(RG) * r * 4, 16); }
size_t roll_lds(int r, bool res) { return RollLds(r, res ? CR_RES : CR_STREAM).total; }

int set_lds(const void* fn, size_t bytes) {
  int dev = 0, maxlds = 0;
  DOPINF_HIP(hipGetDevice(&dev));
  DOPINF_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if (bytes + 1024 > size_t(maxlds)) return fail(DOPINF_E_ARG, "closure needs %zu bytes of LDS, %d available", bytes, maxlds);
  if (bytes > 65536) DOPINF_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
  return DOPINF_OK;
}

}  // namespace
}  // namespace dopinf

using namespace dopinf;

extern "C" int64_t dopinf_closure_param_count(int r) { return (r >= 1 && r <= 64) ? Off(r).P : 0; }

extern "C" int dopinf_rom_residuals(void* stream, const double* O, int r, const double* Qhat, int64_t ldqh, int64_t k,
                                    double* R) {
  DOPINF_REQUIRE(O && Qhat && R, "NULL argument");
  DOPINF_REQUIRE(r >= 1 && r <= 512 && k >= 2 && ldqh >= k, "need 1 <= r <= 512, k >= 2, ldqh >= k");
  const size_t lds = size_t(ncols(r)) * sizeof(double);
  int rc = set_lds(reinterpret_cast<const void*>(residual_kernel), lds);
  if (rc) return rc;
  residual_kernel<<<unsigned(k - 1), 256, lds, static_cast<hipStream_t>(stream)>>>(O, r, Qhat, ldqh, k, R);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}

// the trainer's workgroups exchange gradient shares (one P-vector each, at
// most BMAX / CB workgroups), loss shares and a barrier word through this
// (activations live in LDS)
Carver carve_fit(void* ws, int r, float** gpart, float** lpart, float** img, unsigned** words) {
  Carver c(ws, ~size_t(0));
  *gpart = c.take<float>(size_t(BMAX / CB) * size_t(Off(r).P));
  *lpart = c.take<float>(BMAX / CB);
  *img = c.take<float>(size_t(Img<64>::N));
  *words = c.take<unsigned>(8);
  return c;
}

extern "C" size_t dopinf_closure_fit_workspace(int r, int64_t /*N*/) {
  if (r < 1 || r > 64) return 0;
  float *g, *l, *im;
  unsigned* w;
  return carve_fit(nullptr, r, &g, &l, &im, &w).used;
}

extern "C" int dopinf_closure_fit(void* stream, int r, const double* X, const double* Y, int64_t N, int epochs,
                                  int batch, double lr, double beta1, double beta2, double eps, float* params,
                                  double* norm, float* adam_m, float* adam_v, float* loss_log, void* ws,
                                  size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  DOPINF_REQUIRE(X && Y && params && norm && adam_m && adam_v, "NULL argument");
  DOPINF_REQUIRE(r >= 1 && r <= 64, "closure supports 1 <= r <= 64");
  DOPINF_REQUIRE(N >= 1 && epochs >= 0 && batch >= 1 && batch <= BMAX, "need N >= 1, epochs >= 0, 1 <= batch <= 256");
  DOPINF_REQUIRE(lr > 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0, "invalid Adam settings");
  const size_t need = dopinf_closure_fit_workspace(r, N);
  if (!ws || ws_bytes < need) return fail(DOPINF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const void* kern = r <= 32 ? reinterpret_cast<const void*>(train_kernel<32>)
                             : reinterpret_cast<const void*>(train_kernel<64>);
  int rc = set_lds(kern, train_lds(r));
  if (rc) return rc;
  {
    int dev = 0, coop = 0;
    DOPINF_HIP(hipGetDevice(&dev));
    DOPINF_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return fail(DOPINF_E_HIP, "device does not support cooperative launches");
  }
  TrainArgs a{};
  a.r = r;
  a.X = X;
  a.Y = Y;
  a.N = N;
  a.epochs = epochs;
  a.batch = batch;
  a.lr = float(lr);
  a.beta1 = float(beta1);
  a.beta2 = float(beta2);
  a.eps = float(eps);
  a.params = params;
  a.norm = norm;
  a.m = adam_m;
  a.v = adam_v;
  a.loss_log = loss_log;
  carve_fit(ws, r, &a.Gpart, &a.lpart, &a.img, &a.words);
  zero_u32_kernel<<<1, 64, 0, st>>>(a.words, 8);
  DOPINF_LAUNCHED();
  norm_kernel<<<2 * r, 256, 0, st>>>(X, Y, N, r, norm);
  DOPINF_LAUNCHED();
  const unsigned nw = unsigned((batch + CB - 1) / CB);
  void* args[] = {&a};
  DOPINF_HIP(hipLaunchCooperativeKernel(kern, dim3(nw), dim3(MT), args, unsigned(train_lds(r)), st));
  return DOPINF_OK;
}

extern "C" int dopinf_closure_norms(void* stream, int r, const double* X, const double* Y, int64_t N, double* norm) {
  DOPINF_REQUIRE(X && Y && norm && r >= 1 && r <= 64 && N >= 1, "invalid argument");
  norm_kernel<<<2 * r, 256, 0, static_cast<hipStream_t>(stream)>>>(X, Y, N, r, norm);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}

extern "C" int dopinf_closure_grad(void* stream, int r, const float* params, const double* norm, const double* X,
                                   const double* Y, int64_t N, float* grad, float* loss, void* ws, size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  DOPINF_REQUIRE(params && norm && X && Y && grad && loss, "NULL argument");
  DOPINF_REQUIRE(r >= 1 && r <= 64 && N >= 1 && N <= BMAX, "need 1 <= r <= 64 and 1 <= N <= 256");
  const size_t need = dopinf_closure_fit_workspace(r, N);
  if (!ws || ws_bytes < need) return fail(DOPINF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  const void* kern = r <= 32 ? reinterpret_cast<const void*>(grad_kernel<32>)
                             : reinterpret_cast<const void*>(grad_kernel<64>);
  int rc = set_lds(kern, train_lds(r));
  if (rc) return rc;
  GradArgs a{};
  a.r = r;
  a.X = X;
  a.Y = Y;
  a.N = N;
  a.params = params;
  a.norm = norm;
  a.G = grad;
  a.loss = loss;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (r <= 32)
    grad_kernel<32><<<1, MT, train_lds(r), st>>>(a);
  else
    grad_kernel<64><<<1, MT, train_lds(r), st>>>(a);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}

extern "C" size_t dopinf_closure_eval_workspace(int64_t N) { return N > 0 ? round_up(size_t(N) * 8, 256) : 0; }

extern "C" int dopinf_closure_eval(void* stream, int r, const float* params, const double* norm, const double* X,
                                   int64_t N, double* G, double* gmax, void* ws, size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  DOPINF_REQUIRE(params && norm && X && (G || gmax), "NULL argument");
  DOPINF_REQUIRE(r >= 1 && r <= 64 && N >= 1, "need 1 <= r <= 64, N >= 1");
  if (!ws || ws_bytes < dopinf_closure_eval_workspace(N)) return fail(DOPINF_E_WORKSPACE, "workspace too small");
  int rc = set_lds(reinterpret_cast<const void*>(eval_kernel), eval_lds(r));
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* gn = static_cast<double*>(ws);
  eval_kernel<<<unsigned((N + RG - 1) / RG), ET, eval_lds(r), st>>>(r, params, norm, X, N, G, gn);
  DOPINF_LAUNCHED();
  if (gmax) {
    max_kernel<<<1, 256, 0, st>>>(gn, N, gmax);
    DOPINF_LAUNCHED();
  }
  return DOPINF_OK;
}

extern "C" size_t dopinf_closure_rollout_workspace(int r) { return r > 0 ? round_up(size_t(2 * r) * 8, 256) : 0; }

extern "C" int dopinf_closure_rollout(void* stream, int r, const double* O, const float* params, const double* norm,
                                      double threshold, const double* q0, int64_t M, int n_states, const double* Qref,
                                      int64_t ldref, int64_t k_ref, double max_growth, double* traj, double* err,
                                      double* growth, int* outcome, int* fallback_at, void* ws, size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  DOPINF_REQUIRE(O && q0 && Qref && err && growth && outcome && fallback_at, "NULL argument");
  DOPINF_REQUIRE(threshold <= 0.0 || (params && norm), "params and norm are needed when the closure is on");
  DOPINF_REQUIRE(r >= 1 && r <= 64 && M >= 1 && n_states >= 1 && k_ref >= 1 && ldref >= k_ref && max_growth > 0,
                 "invalid sizes");
  if (!ws || ws_bytes < dopinf_closure_rollout_workspace(r)) return fail(DOPINF_E_WORKSPACE, "workspace too small");
  const bool res = (r <= CW * RES_ROWS) && (ncols(r) <= 64 * RES_NJ);
  const void* kern = res ? reinterpret_cast<const void*>(closure_rollout_kernel<true>)
                         : reinterpret_cast<const void*>(closure_rollout_kernel<false>);
  int rc = set_lds(kern, roll_lds(r, res));
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* mean = static_cast<double*>(ws);
  double* maxdev = mean + r;
  ref_stats_kernel<<<r, 256, 0, st>>>(Qref, ldref, k_ref, mean, maxdev);
  DOPINF_LAUNCHED();
  CRollArgs a{};
  a.r = r;
  a.O = O;
  a.p = params;
  a.norm = norm;
  a.threshold = threshold;
  a.q0 = q0;
  a.M = M;
  a.n_states = n_states;
  a.Qref = Qref;
  a.ldref = ldref;
  a.k_ref = k_ref;
  a.mean = mean;
  a.maxdev = maxdev;
  a.max_growth = max_growth;
  a.traj = traj;
  a.err = err;
  a.growth = growth;
  a.outcome = outcome;
  a.fallback_at = fallback_at;
  if (res)
    closure_rollout_kernel<true><<<unsigned((M + CR_RES - 1) / CR_RES), CT, roll_lds(r, true), st>>>(a);
  else
    closure_rollout_kernel<false><<<unsigned((M + CR_STREAM - 1) / CR_STREAM), CT, roll_lds(r, false), st>>>(a);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}
