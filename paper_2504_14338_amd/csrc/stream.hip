// Out-of-core form of Steps II-III (arXiv:2504.14338, Sec. 3.2 loading and
// Sec. 3.4, Eq. (5)): snapshot matrices that do not fit in device memory stay
// in host memory and stream through two device staging buffers, chunk by
// chunk of rows.  The statistics are per row (means) and per-variable maxima,
// so a chunk's maxima combine by max; the Gram matrix is additive over row
// blocks (Eq. (5)), so each chunk's Gram is added to D in chunk order
// (deterministic).  The host-to-device copy of chunk c+1 runs on a copy
// stream of its own while chunk c's kernels run on the caller's stream:
// two events per buffer (copied / consumed) order the reuse of a buffer.
#include <algorithm>
#include <vector>

#include "common.hpp"

namespace dopinf {
int gram_f64_internal(hipStream_t st, const double* X, int64_t n, int64_t m, int64_t ldx, const double* mean,
                      const double* scale, int nvars, const int64_t* var_rows_h, double* D, int64_t ldd, void* ws,
                      size_t ws_bytes);
size_t gram_f64_workspace_internal(int64_t n, int64_t m, int nvars);
int check_var_rows(int64_t n, int nvars, const int64_t* var_rows_h);

namespace {

// D (+)= P, k x k
__global__ __launch_bounds__(256) void accumulate_kernel(double* __restrict__ D, int64_t ldd,
                                                         const double* __restrict__ P, int64_t k, int first) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= k * k) return;
  const int64_t i = e / k, j = e % k;
  D[i * ldd + j] = first ? P[e] : D[i * ldd + j] + P[e];
}

// max that keeps NaN
__device__ __forceinline__ double max_keep_nan(double a, double b) {
  return (a != a) ? a : ((b != b || b > a) ? b : a);
}

// running per-variable maxima from one chunk: vmax[v0 + j] = max(vmax, chunk
// maximum of local variable j) with a zero-range chunk counting as 0
// (bit j of first_mask: this chunk holds the first rows of local variable j)
__global__ void combine_max_kernel(double* vmax, int v0, int nv, const double* cscale, const int* czr,
                                   unsigned long long first_mask, int* info, const int* cinfo) {
  const int j = threadIdx.x;
  if (j < nv) {
    const double m = czr[j] ? 0.0 : cscale[j];
    vmax[v0 + j] = ((first_mask >> j) & 1ull) ? m : max_keep_nan(vmax[v0 + j], m);
  }
  if (j == 0 && *cinfo != DOPINF_OK) atomicExch(info, *cinfo);
}

__global__ void finalize_scale_kernel(const double* vmax, int nvars, int do_scale, double* scale, int* zero_range) {
  const int v = threadIdx.x;
  if (v >= nvars) return;
  const double m = vmax[v];
  int zr = 0;
  double s = 1.0;
  if (m != m) {
    if (do_scale) s = m;
  } else if (do_scale) {
    if (m == 0.0)
      zr = 1;
    else
      s = m;
  }
  scale[v] = s;
  if (zero_range) zero_range[v] = zr;
}

__global__ void set_ok_kernel(int* p) {
  if (threadIdx.x == 0) *p = DOPINF_OK;
}

struct Chunk {
  int64_t row0, rows;
  int v0, nv;
  std::vector<int64_t> local;  // chunk-local variable boundaries (nv + 1)
};

std::vector<Chunk> make_chunks(int64_t n, int64_t chunk_rows, int nvars, const int64_t* var_rows_h) {
  std::vector<Chunk> out;
  for (int64_t r0 = 0; r0 < n; r0 += chunk_rows) {
    Chunk c;
    c.row0 = r0;
    c.rows = std::min(chunk_rows, n - r0);
    int v0 = 0;
    while (v0 + 1 < nvars && var_rows_h[v0 + 1] <= r0) ++v0;
    int v1 = v0;
    while (v1 + 1 < nvars && var_rows_h[v1 + 1] < r0 + c.rows) ++v1;
    c.v0 = v0;
    c.nv = v1 - v0 + 1;
    c.local.push_back(0);
    for (int v = v0 + 1; v <= v1; ++v) c.local.push_back(var_rows_h[v] - r0);
    c.local.push_back(c.rows);
    out.push_back(std::move(c));
  }
  return out;
}

struct StreamWs {
  double* stage[2];
  double* part;     // k x k chunk Gram (gram) or per-chunk statistics (preprocess)
  double* vmax;     // nvars running maxima
  double* cscale;   // chunk scales
  int* czr;
  int* cinfo;
  void* kws;        // workspace of the per-chunk kernels
  size_t kws_bytes;
};

StreamWs carve_stream(Carver& c, int64_t chunk_rows, int64_t k, int nvars) {
  StreamWs w{};
  w.stage[0] = c.take<double>(size_t(chunk_rows) * k);
  w.stage[1] = c.take<double>(size_t(chunk_rows) * k);
  w.part = c.take<double>(size_t(k) * k);
  w.vmax = c.take<double>(size_t(nvars));
  w.cscale = c.take<double>(size_t(nvars));
  w.czr = c.take<int>(size_t(nvars));
  w.cinfo = c.take<int>(1);
  w.kws_bytes = std::max(gram_f64_workspace_internal(chunk_rows, k, nvars),
                         dopinf_preprocess_workspace(chunk_rows, k, nvars));
  w.kws = c.take<char>(w.kws_bytes);
  return w;
}

// Runs body(chunk index, staged device rows) for every chunk on `st`, with
// the copies on a stream of their own, two buffers deep.
template <class Body>
int run_chunks(hipStream_t st, const double* Q_h, int64_t ldq, int64_t k, const std::vector<Chunk>& chunks,
               const StreamWs& w, Body&& body) {
  hipStream_t cp = nullptr;
  hipEvent_t start = nullptr, copied[2] = {nullptr, nullptr}, consumed[2] = {nullptr, nullptr};
  int rc = DOPINF_OK;
  auto hip_ok = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && !rc) rc = fail(DOPINF_E_HIP, "%s failed: %s", what, hipGetErrorString(e));
    return e == hipSuccess;
  };
  if (hip_ok(hipStreamCreateWithFlags(&cp, hipStreamNonBlocking), "hipStreamCreateWithFlags") &&
      hip_ok(hipEventCreateWithFlags(&start, hipEventDisableTiming), "hipEventCreate") &&
      hip_ok(hipEventCreateWithFlags(&copied[0], hipEventDisableTiming), "hipEventCreate") &&
      hip_ok(hipEventCreateWithFlags(&copied[1], hipEventDisableTiming), "hipEventCreate") &&
      hip_ok(hipEventCreateWithFlags(&consumed[0], hipEventDisableTiming), "hipEventCreate") &&
      hip_ok(hipEventCreateWithFlags(&consumed[1], hipEventDisableTiming), "hipEventCreate")) {
    // the staging buffers may still be in use by earlier work on `st`
    if (hip_ok(hipEventRecord(start, st), "hipEventRecord")) hip_ok(hipStreamWaitEvent(cp, start, 0), "wait");
    for (size_t c = 0; c < chunks.size() && !rc; ++c) {
      const int b = int(c & 1);
      const Chunk& ch = chunks[c];
      if (c >= 2 && !hip_ok(hipStreamWaitEvent(cp, consumed[b], 0), "hipStreamWaitEvent")) break;
      if (!hip_ok(hipMemcpy2DAsync(w.stage[b], size_t(k) * sizeof(double), Q_h + ch.row0 * ldq,
                                   size_t(ldq) * sizeof(double), size_t(k) * sizeof(double), size_t(ch.rows),
                                   hipMemcpyHostToDevice, cp),
                  "hipMemcpy2DAsync"))
        break;
      if (!hip_ok(hipEventRecord(copied[b], cp), "hipEventRecord")) break;
      if (!hip_ok(hipStreamWaitEvent(st, copied[b], 0), "hipStreamWaitEvent")) break;
      const int brc = body(int(c), w.stage[b]);
      if (brc) {
        if (!rc) rc = brc;
        break;
      }
      if (!hip_ok(hipEventRecord(consumed[b], st), "hipEventRecord")) break;
    }
  }
  // the caller's stream does not run past the copies (its kernels waited on
  // every copy); the copy stream and events are released once their work ends
  if (cp) (void)hipStreamDestroy(cp);
  for (hipEvent_t e : {start, copied[0], copied[1], consumed[0], consumed[1]})
    if (e) (void)hipEventDestroy(e);
  return rc;
}

int check_stream_args(const double* Q_h, int64_t n, int64_t k, int64_t ldq, int nvars, const int64_t* var_rows_h,
                      int64_t chunk_rows) {
  DOPINF_REQUIRE(Q_h, "Q_h must be non-NULL");
  DOPINF_REQUIRE(n >= 1 && k >= 1 && ldq >= k, "need n >= 1, k >= 1, ldq >= k");
  DOPINF_REQUIRE(chunk_rows >= 1, "need chunk_rows >= 1");
  return check_var_rows(n, nvars, var_rows_h);
}

}  // namespace
}  // namespace dopinf

using namespace dopinf;

extern "C" size_t dopinf_stream_workspace(int64_t chunk_rows, int64_t k, int nvars) {
  if (chunk_rows <= 0 || k <= 0 || nvars <= 0) return 0;
  Carver c(nullptr, 0);
  carve_stream(c, chunk_rows, k, nvars);
  return c.used;
}

extern "C" int dopinf_preprocess_stream(void* stream, const double* Q_h, int64_t n, int64_t k, int64_t ldq, int nvars,
                                        const int64_t* var_rows_h, unsigned flags, double* mean, double* scale,
                                        int* zero_range, int* info, int64_t chunk_rows, void* ws, size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  int rc = check_stream_args(Q_h, n, k, ldq, nvars, var_rows_h, chunk_rows);
  if (rc) return rc;
  DOPINF_REQUIRE(mean && scale, "mean and scale must be non-NULL");
  DOPINF_REQUIRE((flags & ~(DOPINF_CENTER | DOPINF_SCALE)) == 0, "flags: CENTER and SCALE only (no APPLY)");
  const size_t need = dopinf_stream_workspace(chunk_rows, k, nvars);
  if (!ws || ws_bytes < need) return fail(DOPINF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Carver c(ws, ws_bytes);
  const StreamWs w = carve_stream(c, chunk_rows, k, nvars);
  const std::vector<Chunk> chunks = make_chunks(n, chunk_rows, nvars, var_rows_h);
  if (info) {
    set_ok_kernel<<<1, 64, 0, st>>>(info);
    DOPINF_LAUNCHED();
  }
  // each chunk: per-row means in place, per-variable maxima of the chunk
  // (always with SCALE, so that the maxima can be combined), then the
  // running maxima
  std::vector<int> first_of_var(nvars, 1);
  rc = run_chunks(st, Q_h, ldq, k, chunks, w, [&](int ci, const double* rows) -> int {
    const Chunk& ch = chunks[size_t(ci)];
    int r2 = dopinf_preprocess(st, DOPINF_F64, const_cast<double*>(rows), ch.rows, k, k, ch.nv, ch.local.data(),
                               (flags & DOPINF_CENTER) | DOPINF_SCALE, mean + ch.row0, w.cscale, w.czr, w.cinfo,
                               w.kws, w.kws_bytes);
    if (r2) return r2;
    // a variable's first chunk initializes its running maximum
    unsigned long long first = 0;
    for (int j = 0; j < ch.nv; ++j)
      if (first_of_var[size_t(ch.v0 + j)]) first |= 1ull << j;
    combine_max_kernel<<<1, 64, 0, st>>>(w.vmax, ch.v0, ch.nv, w.cscale, w.czr, first, info ? info : w.cinfo,
                                         w.cinfo);
    DOPINF_LAUNCHED();
    for (int v = ch.v0; v < ch.v0 + ch.nv; ++v) first_of_var[size_t(v)] = 0;
    return DOPINF_OK;
  });
  if (rc) return rc;
  finalize_scale_kernel<<<1, 64, 0, st>>>(w.vmax, nvars, (flags & DOPINF_SCALE) ? 1 : 0, scale, zero_range);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}

extern "C" int dopinf_gram_stream(void* stream, const double* Q_h, int64_t n, int64_t k, int64_t ldq,
                                  const double* mean, const double* scale, int nvars, const int64_t* var_rows_h,
                                  double* D, int64_t ldd, int64_t chunk_rows, void* ws, size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  int rc = check_stream_args(Q_h, n, k, ldq, nvars, var_rows_h, chunk_rows);
  if (rc) return rc;
  DOPINF_REQUIRE(D && ldd >= k, "D must be non-NULL with ldd >= k");
  DOPINF_REQUIRE(k <= (int64_t(1) << 20), "k too large");
  const size_t need = dopinf_stream_workspace(chunk_rows, k, nvars);
  if (!ws || ws_bytes < need) return fail(DOPINF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Carver c(ws, ws_bytes);
  const StreamWs w = carve_stream(c, chunk_rows, k, nvars);
  const std::vector<Chunk> chunks = make_chunks(n, chunk_rows, nvars, var_rows_h);
  return run_chunks(st, Q_h, ldq, k, chunks, w, [&](int ci, const double* rows) -> int {
    const Chunk& ch = chunks[size_t(ci)];
    int r2 = gram_f64_internal(st, rows, ch.rows, k, k, mean ? mean + ch.row0 : nullptr,
                               scale ? scale + ch.v0 : nullptr, scale ? ch.nv : 0,
                               scale ? ch.local.data() : nullptr, w.part, k, w.kws, w.kws_bytes);
    if (r2) return r2;
    accumulate_kernel<<<unsigned((k * k + 255) / 256), 256, 0, st>>>(D, ldd, w.part, k, ci == 0 ? 1 : 0);
    DOPINF_LAUNCHED();
    return DOPINF_OK;
  });
}
