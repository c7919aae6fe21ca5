// Host runtime and C ABI of libellsp2 (see include/ellsp2.h).
//
// Handles own (or borrow) row-major ELLPACK device buffers.  Every argument
// check runs on the host before the first HIP call, so malformed arguments
// are reported without a GPU.  sp2_solve keeps the whole purification loop on
// the device: the per-iteration decision (trace branch, stop, stall, overflow,
// precision switch) is taken on the device by one thread and written to a
// device control block; every kernel of the loop returns at once when that
// block says "stop", and the host reads the block only every poll_every
// iterations.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ellsp2.h"
#include "ell_internal.h"

using namespace ellsp2;

struct ellpack {
  int32_t N = 0, M = 0;
  ell_prec_t prec = ELL_F64;
  bool owned = false;
  bool validated = false;
  int32_t *nnz = nullptr;
  int32_t *idx = nullptr;
  void *val = nullptr;
  hipStream_t stream = nullptr;
};

namespace {
thread_local std::string g_last_error = "no error";
}  // namespace

int ellsp2::device_error(hipError_t e, const char *what)
{
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? ELL_ENOMEM : ELL_EDEVICE;
}

void ellsp2::set_device_error(const char *what) { g_last_error = what; }

namespace {

#define HIP_TRY(expr)                                          \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) return device_error(e_, #expr);      \
  } while (0)

size_t val_size(ell_prec_t p) { return p == ELL_F64 ? sizeof(double) : sizeof(float); }

int32_t roundup32(int64_t x) { return (int32_t)((x + 31) / 32 * 32); }

// Scratch allocations of an API call whose device work all runs on one
// stream (an AllocScope on the call's stack names it) come from a process-wide
// cache of device blocks: repeated calls reuse them instead of paying for
// hipMalloc and a device-synchronising hipFree every time.  A released block
// carries an event recorded on its stream after the work queued before the
// release; a new owner on another stream waits for that event first, so reuse
// is ordered after every earlier use.  The cache holds at most kCacheBytes
// (oldest blocks are freed beyond that).  Without a scope, allocations are
// plain hipMalloc / hipFree; a scope opened with cache = false keeps them so
// but still names the stream their fills are queued on (a call whose work runs
// on a non-blocking stream, which does not wait for the null stream).
thread_local bool g_cache_alloc = false;
thread_local hipStream_t g_cache_stream = nullptr;

struct CachedBlock {
  void *p;
  size_t bytes;
  int dev;
  hipStream_t stream;
  hipEvent_t done;
};
constexpr size_t kCacheBytes = (size_t)16 << 30;
std::mutex g_cache_mu;
std::vector<CachedBlock> g_cache;
size_t g_cache_total = 0;

size_t size_class(size_t bytes)
{
  const size_t g = bytes >= ((size_t)1 << 20) ? ((size_t)1 << 16) : 256;  // 64 KiB steps above 1 MiB
  return (std::max<size_t>(bytes, 1) + g - 1) / g * g;
}

struct AllocScope {
  bool prev_on;
  hipStream_t prev_stream;
  explicit AllocScope(hipStream_t s, bool cache = true) : prev_on(g_cache_alloc), prev_stream(g_cache_stream)
  {
    g_cache_alloc = cache;
    g_cache_stream = s;
  }
  ~AllocScope()
  {
    g_cache_alloc = prev_on;
    g_cache_stream = prev_stream;
  }
  AllocScope(const AllocScope &) = delete;
  AllocScope &operator=(const AllocScope &) = delete;
};

// Device allocation released on scope exit.
struct DevMem {
  void *p = nullptr;
  bool cached = false;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;  // the block's reuse event (cached blocks)
  size_t bytes = 0;
  int dev = 0;
  DevMem() = default;
  DevMem(const DevMem &) = delete;
  DevMem &operator=(const DevMem &) = delete;
  ~DevMem() { release(); }
  void release()
  {
    if (!p) return;
    if (!cached) {
      (void)hipFree(p);
    } else if (!done && hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamSynchronize(stream);
      (void)hipFree(p);
    } else {
      (void)hipEventRecord(done, stream);
      std::vector<CachedBlock> evict;
      {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        g_cache.push_back(CachedBlock{p, bytes, dev, stream, done});
        g_cache_total += bytes;
        while (g_cache_total > kCacheBytes && !g_cache.empty()) {
          evict.push_back(g_cache.front());
          g_cache_total -= g_cache.front().bytes;
          g_cache.erase(g_cache.begin());
        }
      }
      for (const CachedBlock &c : evict) {
        (void)hipEventSynchronize(c.done);
        (void)hipEventDestroy(c.done);
        (void)hipFree(c.p);
      }
    }
    p = nullptr;
    done = nullptr;
  }
  hipError_t alloc(size_t want)
  {
    release();
    cached = g_cache_alloc;
    stream = g_cache_stream;
    if (!cached) return hipMalloc(&p, want ? want : 1);
    bytes = size_class(want);
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    {
      std::lock_guard<std::mutex> lock(g_cache_mu);
      for (size_t i = g_cache.size(); i-- > 0;) {
        const CachedBlock &c = g_cache[i];
        if (c.dev == dev && c.bytes == bytes) {
          p = c.p;
          done = c.done;
          const hipStream_t from = c.stream;
          g_cache_total -= c.bytes;
          g_cache.erase(g_cache.begin() + (ptrdiff_t)i);
          return from == stream ? hipSuccess : hipStreamWaitEvent(stream, done, 0);
        }
      }
    }
    return hipMalloc(&p, bytes);
  }
  template <typename T>
  T *as() const { return static_cast<T *>(p); }
  // fills are queued on the scope's stream (or, outside any scope, are plain hipMemset)
  bool ordered() const { return cached || stream; }
  // zero the first `n` bytes, ordered like the allocation
  hipError_t zero(size_t n) const { return ordered() ? hipMemsetAsync(p, 0, n, stream) : hipMemset(p, 0, n); }
};

void swap_mem(DevMem &a, DevMem &b)
{
  std::swap(a.p, b.p);
  std::swap(a.cached, b.cached);
  std::swap(a.stream, b.stream);
  std::swap(a.done, b.done);
  std::swap(a.bytes, b.bytes);
  std::swap(a.dev, b.dev);
}

// Pinned, device-mapped, coherent host blocks (the SP2 loop's state slots, its
// initialisation results, its history) come from a small process-wide pool,
// so a solve does not pay for hipHostMalloc every time.  A block returns to
// the pool only after its stream has drained (no kernel still writes it).
struct PinnedBlock {
  void *p;
  void *d;  // the device's address of it
  size_t bytes;
};
constexpr size_t kPinnedPoolBlocks = 16;
std::mutex g_pin_mu;
std::vector<PinnedBlock> g_pin_pool;

struct PinnedMem {
  PinnedBlock b{nullptr, nullptr, 0};
  PinnedMem() = default;
  PinnedMem(const PinnedMem &) = delete;
  PinnedMem &operator=(const PinnedMem &) = delete;
  ~PinnedMem() { release(); }
  void release()
  {
    if (!b.p) return;
    {
      std::lock_guard<std::mutex> lock(g_pin_mu);
      if (g_pin_pool.size() < kPinnedPoolBlocks) {
        g_pin_pool.push_back(b);
        b = PinnedBlock{nullptr, nullptr, 0};
        return;
      }
    }
    (void)hipHostFree(b.p);
    b = PinnedBlock{nullptr, nullptr, 0};
  }
  hipError_t alloc(size_t want)
  {
    release();
    const size_t bytes = size_class(want);
    {
      std::lock_guard<std::mutex> lock(g_pin_mu);
      for (size_t i = g_pin_pool.size(); i-- > 0;)
        if (g_pin_pool[i].bytes == bytes) {
          b = g_pin_pool[i];
          g_pin_pool.erase(g_pin_pool.begin() + (ptrdiff_t)i);
          return hipSuccess;
        }
    }
    void *h = nullptr, *d = nullptr;
    hipError_t e = hipHostMalloc(&h, bytes, hipHostMallocMapped | hipHostMallocCoherent | hipHostMallocPortable);
    if (e != hipSuccess) return e;
    e = hipHostGetDevicePointer(&d, h, 0);
    if (e != hipSuccess) {
      (void)hipHostFree(h);
      return e;
    }
    b = PinnedBlock{h, d, bytes};
    return hipSuccess;
  }
  template <typename T>
  T *host(size_t off) const { return reinterpret_cast<T *>(static_cast<char *>(b.p) + off); }
  template <typename T>
  T *dev(size_t off) const { return reinterpret_cast<T *>(static_cast<char *>(b.d) + off); }
};

int have_device()
{
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) {
    g_last_error = "no HIP device available";
    return ELL_ENODEV;
  }
  return ELL_OK;
}

template <typename T>
EllView<T> view(const ellpack *A)
{
  return EllView<T>{A->nnz, A->idx, static_cast<T *>(A->val), A->M};
}

template <typename T>
int validate_on_device(const ellpack *A_)
{
  ellpack *A = const_cast<ellpack *>(A_);
  if (A->validated) return ELL_OK;
  AllocScope scope(A->stream);
  DevMem flags;
  HIP_TRY(flags.alloc(sizeof(int32_t)));
  HIP_TRY(hipMemsetAsync(flags.p, 0, sizeof(int32_t), A->stream));
  HIP_TRY(launch_validate<T>(A->N, view<T>(A), flags.as<int32_t>(), A->stream));
  int32_t h = 0;
  HIP_TRY(hipMemcpyAsync(&h, flags.p, sizeof(h), hipMemcpyDeviceToHost, A->stream));
  HIP_TRY(hipStreamSynchronize(A->stream));
  if (h & 1) return ELL_EINVAL;
  if (h & 2) return ELL_ENONFINITE;
  A->validated = true;
  return ELL_OK;
}

int ensure_valid(const ellpack *A)
{
  return A->prec == ELL_F64 ? validate_on_device<double>(A) : validate_on_device<float>(A);
}

// Scratch of one fused step for N rows.
struct StepMem {
  DevMem d1, d2, e, wy, wu, ly, lu, part, partw, partn, out, outw, outn, flags;  // flags: the flag, then the ticket
  StepScratch s{};
  hipError_t alloc(int N)
  {
    const int nb = (N + kRedBlock - 1) / kRedBlock;
    const int nq = (N + 63) / 64;  // 64-row partials of the matrix-core span iteration; nq >= nb
    int lq = 1;                    // leaves per thread of the 256-thread trees over them
    while (256 * lq < nq) lq *= 2;
    hipError_t err;
    if ((err = d1.alloc(sizeof(double) * N)) || (err = d2.alloc(sizeof(double) * N)) ||
        (err = e.alloc(sizeof(double) * N)) || (err = wy.alloc(sizeof(int32_t) * N)) ||
        (err = wu.alloc(sizeof(int32_t) * N)) || (err = ly.alloc(sizeof(int32_t) * N)) ||
        (err = lu.alloc(sizeof(int32_t) * N)) || (err = part.alloc(sizeof(double) * (5 * nq + 256 * lq))) ||
        (err = partw.alloc(sizeof(int32_t) * 4 * nq)) || (err = partn.alloc(sizeof(int64_t) * 2 * nq)) ||
        (err = out.alloc(sizeof(double) * 5)) || (err = outw.alloc(sizeof(int32_t) * 4)) ||
        (err = outn.alloc(sizeof(int64_t) * 2)) || (err = flags.alloc(2 * sizeof(int32_t))))
      return err;
    if ((err = flags.zero(2 * sizeof(int32_t)))) return err;  // the fallback flag, then the ticket
    s.d1 = d1.as<double>();
    s.d2 = d2.as<double>();
    s.e = e.as<double>();
    s.wy = wy.as<int32_t>();
    s.wu = wu.as<int32_t>();
    s.ly = ly.as<int32_t>();
    s.lu = lu.as<int32_t>();
    s.flags = flags.as<int32_t>();
    s.ticket = reinterpret_cast<uint32_t *>(flags.as<int32_t>() + 1);
    s.part = part.as<double>();
    s.partw = partw.as<int32_t>();
    s.partn = partn.as<int64_t>();
    s.out = out.as<double>();
    s.outw = outw.as<int32_t>();
    s.outn = outn.as<int64_t>();
    s.nb = nb;
    s.nq = nq;
    return hipSuccess;
  }
};

bool bad_tau(double tau) { return !(tau >= 0.0); }  // rejects NaN and negatives

// The ELLPACK pipeline neither writes interval lengths nor raises the fallback flag.
StepScratch ell_scratch(const StepScratch &s)
{
  StepScratch t = s;
  t.ly = t.lu = nullptr;
  t.flags = nullptr;
  return t;
}

int32_t roundup64(int64_t x) { return (int32_t)((x + 63) / 64 * 64); }

// Span-form storage of one matrix (see SpanView).
template <typename T>
struct SpanMem {
  DevMem val, base, len;
  int32_t SW = 0;
  // zero_values: false when only the symmetric iteration reads the matrices
  // (its reads stay inside the row intervals, which every writer fills)
  // zero_intervals false: the caller clears base and len (several matrices' in one launch)
  hipError_t alloc(int N, int32_t sw, bool zero_values = true, bool zero_intervals = true)
  {
    SW = sw;
    hipError_t e;
    if ((e = val.alloc(sizeof(T) * ((size_t)N * sw + 2 * kSpanGuard))) ||
        (e = base.alloc(sizeof(int32_t) * ((size_t)N + kSpanPadRows))) ||
        (e = len.alloc(sizeof(int32_t) * ((size_t)N + kSpanPadRows))))
      return e;
    // rows past N read as empty by the band kernel's batched interval loads
    if (zero_intervals) {
      if ((e = base.zero(sizeof(int32_t) * ((size_t)N + kSpanPadRows)))) return e;
      if ((e = len.zero(sizeof(int32_t) * ((size_t)N + kSpanPadRows)))) return e;
    }
    // the guard bands are read (and masked) by the band kernel: keep them finite
    return zero_values ? val.zero(sizeof(T) * ((size_t)N * sw + 2 * kSpanGuard)) : hipSuccess;
  }
  void release()
  {
    val.release();
    base.release();
    len.release();
    SW = 0;
  }
  SpanView<T> v() const
  {
    return SpanView<T>{val.as<T>() + kSpanGuard, base.as<int32_t>(), len.as<int32_t>(), SW};
  }
};

// Longest row interval of an ELLPACK matrix, whether it stores exact zeros,
// and whether its rows fill their intervals densely enough for span form.
template <typename T>
int ell_extent(const ellpack *A, DevMem &lens, int32_t *maxlen, bool *zeros, bool *dense = nullptr)
{
  struct Ext {
    int32_t flags, maxlen;
    unsigned long long sums[2];
  };
  DevMem ex;
  HIP_TRY(lens.alloc(sizeof(int32_t) * A->N));
  HIP_TRY(ex.alloc(sizeof(Ext)));
  HIP_TRY(hipMemsetAsync(ex.p, 0, sizeof(Ext), A->stream));
  Ext *e = ex.as<Ext>();
  HIP_TRY(launch_ell_extent<T>(A->N, view<T>(A), lens.as<int32_t>(), &e->flags, &e->maxlen, e->sums, A->stream));
  Ext h{};
  HIP_TRY(hipMemcpyAsync(&h, ex.p, sizeof(Ext), hipMemcpyDeviceToHost, A->stream));
  HIP_TRY(hipStreamSynchronize(A->stream));
  *maxlen = h.maxlen;
  *zeros = (h.flags & 4) != 0;
  if (dense) *dense = (unsigned long long)kMinSpanFillInv * h.sums[0] >= h.sums[1];
  return ELL_OK;
}

template <typename T>
int finish_step(const ellpack *X, ellpack *Y, ellpack *U, const StepMem &m, double out[3], int32_t widths[2])
{
  double h[3];
  int32_t w[4];
  HIP_TRY(hipMemcpyAsync(h, m.s.out, sizeof(h), hipMemcpyDeviceToHost, X->stream));
  HIP_TRY(hipMemcpyAsync(w, m.s.outw, sizeof(w), hipMemcpyDeviceToHost, X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  if (out) {
    out[0] = h[0];
    out[1] = h[1];
    out[2] = h[2];
  }
  if (widths) {
    widths[0] = w[0];
    widths[1] = U ? w[1] : 0;
  }
  const bool over = w[0] > Y->M || (U && w[1] > U->M);
  if (over) return ELL_EOVERFLOW;
  Y->validated = true;
  if (U) U->validated = true;
  return ELL_OK;
}

// Step through the matrix-core band kernel: span form in and out, then the
// rows of X^2 and 2X - X^2 compacted into the ELLPACK outputs.  Returns
// kNotTaken (nothing written to Y or U) when a row group's window or an output
// interval does not fit the span stride.
constexpr int kNotTaken = 1;
template <typename T>
int run_step_band16(const ellpack *X, ellpack *Y, ellpack *U, double tau, int32_t maxlen, StepMem &m, double out[3],
                    int32_t widths[2])
{
  const int N = X->N;
  const int32_t sw = std::max<int32_t>(256, roundup64(std::min<int64_t>(N, 3 * (int64_t)maxlen)));
  if (!x2_band16_fits(N, sw, (int)sizeof(T))) return kNotTaken;
  SpanMem<T> sx, sy, su;
  HIP_TRY(sx.alloc(N, sw));
  HIP_TRY(sy.alloc(N, sw));
  if (U) HIP_TRY(su.alloc(N, sw));
  HIP_TRY(launch_ell_to_span<T>(N, view<T>(X), sx.v(), X->stream));
  // X^2 to slot 1, 2X - X^2 to slot 2 (without U: X^2 alone, slot 2 untouched)
  const SpanRot3<T> spans{{sx.v(), sy.v(), U ? su.v() : sy.v()}};
  HIP_TRY(launch_x2_band16<T>(N, spans, nullptr, (T)tau, m.s, m.s.flags, X->stream, U != nullptr));
  HIP_TRY(launch_reduce(N, nullptr, m.s, X->stream));
  HIP_TRY(launch_final_only(m.s, X->stream));
  int32_t fb = 0, w[4];
  HIP_TRY(hipMemcpyAsync(&fb, m.s.flags, sizeof(fb), hipMemcpyDeviceToHost, X->stream));
  HIP_TRY(hipMemcpyAsync(w, m.s.outw, sizeof(w), hipMemcpyDeviceToHost, X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  if ((fb & 1) || w[2] > sw || w[3] > sw) {
    HIP_TRY(hipMemsetAsync(m.s.flags, 0, sizeof(int32_t), X->stream));
    return kNotTaken;
  }
  HIP_TRY((launch_span_to_ell<T, T>(N, sy.v(), view<T>(Y), nullptr, X->stream)));
  if (U) HIP_TRY((launch_span_to_ell<T, T>(N, su.v(), view<T>(U), nullptr, X->stream)));
  return finish_step<T>(X, Y, U, m, out, widths);
}

// One fused step on ELLPACK handles.  Matrices whose rows are short intervals
// go through a band kernel after an exact conversion to span form (the
// matrix-core kernel when the span matrices fit its 2^31-byte buffer range,
// else the register-tiled one, which hands row groups with too wide a window
// on); anything else through the LDS-window kernel.
template <typename T>
int run_step(const ellpack *X, ellpack *Y, ellpack *U, double tau, double out[3], int32_t widths[2])
{
  const int N = X->N;
  AllocScope scope(X->stream);
  StepMem m;
  HIP_TRY(m.alloc(N));
  Rot3<T> bufs{{view<T>(X), view<T>(Y), U ? view<T>(U) : view<T>(Y)}};
  DevMem lens;
  int32_t maxlen = 0;
  bool zeros = false, dense = false;
  int rc = ell_extent<T>(X, lens, &maxlen, &zeros, &dense);
  if (rc) return rc;
  if (!zeros && dense && maxlen <= kMaxCap) {
    rc = run_step_band16<T>(X, Y, U, tau, maxlen, m, out, widths);
    if (rc != kNotTaken) return rc;
    SpanMem<T> sx;
    HIP_TRY(sx.alloc(N, std::max(64, roundup64(maxlen))));
    HIP_TRY(launch_ell_to_span<T>(N, view<T>(X), sx.v(), X->stream));
    SpanRot3<T> spans{{sx.v(), sx.v(), sx.v()}};  // outputs go to ELLPACK; the span slots are unused
    HIP_TRY(launch_x2_band<T>(N, spans, bufs, nullptr, U != nullptr, true, (T)tau, m.s, m.s.flags, X->stream));
    int32_t fb = 0;
    HIP_TRY(hipMemcpyAsync(&fb, m.s.flags, sizeof(fb), hipMemcpyDeviceToHost, X->stream));
    HIP_TRY(hipStreamSynchronize(X->stream));
    if (!(fb & 1)) {
      HIP_TRY(launch_reduce(N, nullptr, m.s, X->stream));
      HIP_TRY(launch_final_only(m.s, X->stream));
      return finish_step<T>(X, Y, U, m, out, widths);
    }
  }
  const StepScratch se = ell_scratch(m.s);
  if (!dense) {
    // rows that fill little of their column intervals: the hashed accumulator,
    // then the window kernel for rows with too many products for its table
    DevMem left, nleft;
    HIP_TRY(left.alloc(sizeof(int32_t) * N));
    HIP_TRY(nleft.alloc(sizeof(int32_t)));
    HIP_TRY(launch_x2_hash<T>(N, bufs, U != nullptr, (T)tau, se, left.as<int32_t>(), nleft.as<int32_t>(),
                              X->stream));
  } else {
    HIP_TRY(launch_x2_step<T>(N, bufs, nullptr, U != nullptr, (T)tau, se, X->stream));
  }
  HIP_TRY(launch_reduce(N, nullptr, se, X->stream));
  HIP_TRY(launch_final_only(se, X->stream));
  return finish_step<T>(X, Y, U, m, out, widths);
}

int check_step_args(const ellpack *X, const ellpack *Y, const ellpack *U, double tau)
{
  if (!X || !Y) return ELL_EINVAL;
  if (X == Y || (U && (U == X || U == Y))) return ELL_EINVAL;
  if (X->N != Y->N || X->prec != Y->prec) return ELL_EINVAL;
  if (U && (U->N != X->N || U->prec != X->prec)) return ELL_EINVAL;
  if (X->val == Y->val || (U && (U->val == X->val || U->val == Y->val))) return ELL_EINVAL;
  if (bad_tau(tau)) return ELL_EINVAL;
  return ELL_OK;
}

}  // namespace

// ===========================================================================
// handles
// ===========================================================================
extern "C" int ellpack_check_host(int32_t N, int32_t M, const int32_t *nnz, const int32_t *index,
                                  const double *value)
{
  if (N <= 0 || N > kMaxN || M <= 0 || M > kMaxCap || !nnz || !index) return ELL_EINVAL;
  for (int32_t i = 0; i < N; ++i) {
    if (nnz[i] < 0 || nnz[i] > M) return ELL_EINVAL;
    const int32_t *c = index + (int64_t)i * M;
    for (int32_t q = 0; q < nnz[i]; ++q) {
      if (c[q] < 0 || c[q] >= N) return ELL_EINVAL;
      if (q > 0 && c[q] <= c[q - 1]) return ELL_EINVAL;
    }
  }
  if (value)
    for (int32_t i = 0; i < N; ++i)
      for (int32_t q = 0; q < nnz[i]; ++q)
        if (!std::isfinite(value[(int64_t)i * M + q])) return ELL_ENONFINITE;
  return ELL_OK;
}

extern "C" int ellpack_alloc(ellpack_t **A, int32_t N, int32_t M, ell_prec_t prec, void *hip_stream)
{
  if (!A || N <= 0 || N > kMaxN || M <= 0 || M > kMaxCap || (prec != ELL_F64 && prec != ELL_F32))
    return ELL_EINVAL;
  *A = nullptr;
  int rc = have_device();
  if (rc) return rc;
  ellpack *h = new (std::nothrow) ellpack;
  if (!h) return ELL_ENOMEM;
  h->N = N;
  h->M = M;
  h->prec = prec;
  h->owned = true;
  h->stream = static_cast<hipStream_t>(hip_stream);
  const size_t slots = (size_t)N * M;
  hipError_t e = hipMalloc(&h->nnz, sizeof(int32_t) * N);
  if (e == hipSuccess) e = hipMalloc(&h->idx, sizeof(int32_t) * slots);
  if (e == hipSuccess) e = hipMalloc(&h->val, val_size(prec) * slots);
  if (e == hipSuccess) e = hipMemsetAsync(h->nnz, 0, sizeof(int32_t) * N, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    int r = device_error(e, "ellpack_alloc");
    ellpack_free(h);
    return r;
  }
  h->validated = true;
  *A = h;
  return ELL_OK;
}

extern "C" int ellpack_wrap(ellpack_t **A, int32_t N, int32_t M, ell_prec_t prec, int32_t *d_nnz,
                            int32_t *d_index, void *d_value, void *hip_stream)
{
  if (!A || N <= 0 || N > kMaxN || M <= 0 || M > kMaxCap || !d_nnz || !d_index || !d_value) return ELL_EINVAL;
  if (prec != ELL_F64 && prec != ELL_F32) return ELL_EINVAL;
  *A = nullptr;
  ellpack *h = new (std::nothrow) ellpack;
  if (!h) return ELL_ENOMEM;
  h->N = N;
  h->M = M;
  h->prec = prec;
  h->owned = false;
  h->validated = false;
  h->nnz = d_nnz;
  h->idx = d_index;
  h->val = d_value;
  h->stream = static_cast<hipStream_t>(hip_stream);
  *A = h;
  return ELL_OK;
}

extern "C" int ellpack_free(ellpack_t *A)
{
  if (!A) return ELL_OK;
  if (A->owned) {
    if (A->nnz) (void)hipFree(A->nnz);
    if (A->idx) (void)hipFree(A->idx);
    if (A->val) (void)hipFree(A->val);
  }
  delete A;
  return ELL_OK;
}

extern "C" int ellpack_info(const ellpack_t *A, int32_t *N, int32_t *M, int32_t *prec)
{
  if (!A) return ELL_EINVAL;
  if (N) *N = A->N;
  if (M) *M = A->M;
  if (prec) *prec = (int32_t)A->prec;
  return ELL_OK;
}

extern "C" int ellpack_upload(ellpack_t *A, const int32_t *nnz, const int32_t *index, const double *value)
{
  if (!A || !value) return ELL_EINVAL;
  int rc = ellpack_check_host(A->N, A->M, nnz, index, value);
  if (rc) return rc;
  const size_t slots = (size_t)A->N * A->M;
  HIP_TRY(hipMemcpyAsync(A->nnz, nnz, sizeof(int32_t) * A->N, hipMemcpyHostToDevice, A->stream));
  HIP_TRY(hipMemcpyAsync(A->idx, index, sizeof(int32_t) * slots, hipMemcpyHostToDevice, A->stream));
  if (A->prec == ELL_F64) {
    HIP_TRY(hipMemcpyAsync(A->val, value, sizeof(double) * slots, hipMemcpyHostToDevice, A->stream));
    HIP_TRY(hipStreamSynchronize(A->stream));
  } else {
    std::vector<float> f(slots);
    for (size_t q = 0; q < slots; ++q) f[q] = (float)value[q];
    HIP_TRY(hipMemcpyAsync(A->val, f.data(), sizeof(float) * slots, hipMemcpyHostToDevice, A->stream));
    HIP_TRY(hipStreamSynchronize(A->stream));
  }
  A->validated = true;
  return ELL_OK;
}

extern "C" int ellpack_download(const ellpack_t *A, int32_t *nnz, int32_t *index, double *value)
{
  if (!A || !nnz || !index || !value) return ELL_EINVAL;
  const size_t slots = (size_t)A->N * A->M;
  HIP_TRY(hipMemcpyAsync(nnz, A->nnz, sizeof(int32_t) * A->N, hipMemcpyDeviceToHost, A->stream));
  HIP_TRY(hipMemcpyAsync(index, A->idx, sizeof(int32_t) * slots, hipMemcpyDeviceToHost, A->stream));
  std::vector<float> f;
  if (A->prec == ELL_F64) {
    HIP_TRY(hipMemcpyAsync(value, A->val, sizeof(double) * slots, hipMemcpyDeviceToHost, A->stream));
  } else {
    f.resize(slots);
    HIP_TRY(hipMemcpyAsync(f.data(), A->val, sizeof(float) * slots, hipMemcpyDeviceToHost, A->stream));
  }
  HIP_TRY(hipStreamSynchronize(A->stream));
  for (int32_t i = 0; i < A->N; ++i) {
    const int32_t n = std::min(std::max(nnz[i], 0), A->M);
    for (int32_t q = 0; q < A->M; ++q) {
      const size_t at = (size_t)i * A->M + q;
      if (q >= n) {
        index[at] = -1;
        value[at] = 0.0;
      } else if (A->prec == ELL_F32) {
        value[at] = (double)f[at];
      }
    }
  }
  return ELL_OK;
}

// ===========================================================================
// single operations
// ===========================================================================
extern "C" int ellpack_x2_step(const ellpack_t *X, ellpack_t *X2, ellpack_t *U, double tau, double out[3],
                               int32_t widths[2])
{
  int rc = check_step_args(X, X2, U, tau);
  if (rc) return rc;
  rc = ensure_valid(X);
  if (rc) return rc;
  return X->prec == ELL_F64 ? run_step<double>(X, X2, U, tau, out, widths)
                            : run_step<float>(X, X2, U, tau, out, widths);
}

extern "C" int ellpack_x2_threshold(const ellpack_t *X, ellpack_t *X2, double tau, double trace_out[2],
                                    int32_t *max_row_width_out)
{
  double out[3];
  int32_t w[2] = {0, 0};
  int rc = ellpack_x2_step(X, X2, nullptr, tau, out, w);
  if (rc == ELL_OK || rc == ELL_EOVERFLOW) {
    if (trace_out) {
      trace_out[0] = out[0];
      trace_out[1] = out[1];
    }
    if (max_row_width_out) *max_row_width_out = w[0];
  }
  return rc;
}

// ===========================================================================
// the fused step without allocation
// ===========================================================================
namespace {

// Scratch of ellpack_x2_step_noalloc: the per-row outputs and reduction
// partials of the ELLPACK step kernel for up to kNoAllocMaxN rows, in one
// file-scope device array (each device holds its own copy until the process
// ends).  Layout, every part starting on a 256-byte boundary:
//   [0, 256)           validation flag (int32), out (3 double), outw (4 int32), outn (2 int64)
//   part   3 nb double, partw 4 nb int32, partn 2 nb int64   (nb = ceil(N / 1024) <= kNoAllocBlocks)
//   d1, d2, e          kNoAllocMaxN double each
//   wy, wu             kNoAllocMaxN int32 each
constexpr int32_t kNoAllocMaxN = 131072;
constexpr int32_t kNoAllocBlocks = (kNoAllocMaxN + kRedBlock - 1) / kRedBlock;
constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t kNaHead = 0;
constexpr size_t kNaPart = 256;
constexpr size_t kNaPartW = kNaPart + align256(sizeof(double) * 3 * kNoAllocBlocks);
constexpr size_t kNaPartN = kNaPartW + align256(sizeof(int32_t) * 4 * kNoAllocBlocks);
constexpr size_t kNaRows = kNaPartN + align256(sizeof(int64_t) * 2 * kNoAllocBlocks);
constexpr size_t kNaD1 = kNaRows;
constexpr size_t kNaD2 = kNaD1 + align256(sizeof(double) * kNoAllocMaxN);
constexpr size_t kNaE = kNaD2 + align256(sizeof(double) * kNoAllocMaxN);
constexpr size_t kNaWy = kNaE + align256(sizeof(double) * kNoAllocMaxN);
constexpr size_t kNaWu = kNaWy + align256(sizeof(int32_t) * kNoAllocMaxN);
constexpr size_t kNoAllocBytes = kNaWu + align256(sizeof(int32_t) * kNoAllocMaxN);  // about 4 MiB

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Device address of `scratch` on each device, resolved once per device with
// that device current.  In host code the array's name is only a host-side
// stand-in: kernels receive these addresses.
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_noalloc_mu;
unsigned char *g_noalloc_ptr[kNoAllocMaxDevices] = {};

int noalloc_scratch(unsigned char **out)
{
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices) {
    set_device_error("ellpack_x2_step_noalloc: device ordinal beyond the library's table of 64");
    return ELL_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_device_error("ellpack_x2_step_noalloc: no device address for the scratch array");
      return ELL_EDEVICE;
    }
    g_noalloc_ptr[dev] = static_cast<unsigned char *>(p);
  }
  *out = g_noalloc_ptr[dev];
  return ELL_OK;
}

template <typename T>
int run_step_noalloc(const ellpack *X, ellpack *Y, ellpack *U, double tau, double out[3], int32_t widths[2])
{
  const int N = X->N;
  unsigned char *base = nullptr;
  int rc = noalloc_scratch(&base);
  if (rc) return rc;
  int32_t *flag = reinterpret_cast<int32_t *>(base + kNaHead);
  StepScratch s{};
  s.out = reinterpret_cast<double *>(base + kNaHead + 64);
  s.outw = reinterpret_cast<int32_t *>(base + kNaHead + 128);
  s.outn = reinterpret_cast<int64_t *>(base + kNaHead + 192);
  s.part = reinterpret_cast<double *>(base + kNaPart);
  s.partw = reinterpret_cast<int32_t *>(base + kNaPartW);
  s.partn = reinterpret_cast<int64_t *>(base + kNaPartN);
  s.d1 = reinterpret_cast<double *>(base + kNaD1);
  s.d2 = reinterpret_cast<double *>(base + kNaD2);
  s.e = reinterpret_cast<double *>(base + kNaE);
  s.wy = reinterpret_cast<int32_t *>(base + kNaWy);
  s.wu = reinterpret_cast<int32_t *>(base + kNaWu);
  s.ly = s.lu = nullptr;
  s.flags = nullptr;
  s.nb = (N + kRedBlock - 1) / kRedBlock;
  s.nq = (N + 63) / 64;
  // a wrapped X is validated on its first use, as by ellpack_x2_step, with
  // the flag in the scratch array (cleared first: it keeps the last call's value)
  if (!X->validated) {
    HIP_TRY(launch_zero_words(1, flag, X->stream));
    HIP_TRY(launch_validate<T>(N, view<T>(X), flag, X->stream));
    int32_t h = 0;
    HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, X->stream));
    HIP_TRY(hipStreamSynchronize(X->stream));
    if (h & 1) return ELL_EINVAL;
    if (h & 2) return ELL_ENONFINITE;
    const_cast<ellpack *>(X)->validated = true;
  }
  Rot3<T> bufs{{view<T>(X), view<T>(Y), U ? view<T>(U) : view<T>(Y)}};
  HIP_TRY(launch_x2_step<T>(N, bufs, nullptr, U != nullptr, (T)tau, s, X->stream));
  HIP_TRY(launch_reduce(N, nullptr, s, X->stream));
  HIP_TRY(launch_final_only(s, X->stream));
  double h[3];
  int32_t w[4];
  HIP_TRY(hipMemcpyAsync(h, s.out, sizeof(h), hipMemcpyDeviceToHost, X->stream));
  HIP_TRY(hipMemcpyAsync(w, s.outw, sizeof(w), hipMemcpyDeviceToHost, X->stream));
  HIP_TRY(hipStreamSynchronize(X->stream));
  if (out) {
    out[0] = h[0];
    out[1] = h[1];
    out[2] = h[2];
  }
  if (widths) {
    widths[0] = w[0];
    widths[1] = U ? w[1] : 0;
  }
  if (w[0] > Y->M || (U && w[1] > U->M)) return ELL_EOVERFLOW;
  Y->validated = true;
  if (U) U->validated = true;
  return ELL_OK;
}

}  // namespace

extern "C" int ellpack_x2_step_noalloc(const ellpack_t *X, ellpack_t *X2, ellpack_t *U, double tau, double out[3],
                                       int32_t widths[2])
{
  int rc = check_step_args(X, X2, U, tau);
  if (rc) return rc;
  if (X->N > kNoAllocMaxN) {
    g_last_error = "ellpack_x2_step_noalloc: N exceeds the 131072 rows of its fixed scratch";
    return ELL_EINVAL;
  }
  return X->prec == ELL_F64 ? run_step_noalloc<double>(X, X2, U, tau, out, widths)
                            : run_step_noalloc<float>(X, X2, U, tau, out, widths);
}

extern "C" int ellpack_trace(const ellpack_t *A, double *trace_out)
{
  if (!A || !trace_out) return ELL_EINVAL;
  int rc = ensure_valid(A);
  if (rc) return rc;
  AllocScope scope(A->stream);
  DevMem d, part, out;
  HIP_TRY(d.alloc(sizeof(double) * A->N));
  HIP_TRY(part.alloc(sizeof(double) * ((A->N + kRedBlock - 1) / kRedBlock)));
  HIP_TRY(out.alloc(sizeof(double)));
  if (A->prec == ELL_F64)
    HIP_TRY(launch_trace_rows<double>(A->N, view<double>(A), d.as<double>(), A->stream));
  else
    HIP_TRY(launch_trace_rows<float>(A->N, view<float>(A), d.as<double>(), A->stream));
  HIP_TRY(launch_tree_sum(A->N, d.as<double>(), part.as<double>(), out.as<double>(), A->stream));
  HIP_TRY(hipMemcpyAsync(trace_out, out.p, sizeof(double), hipMemcpyDeviceToHost, A->stream));
  HIP_TRY(hipStreamSynchronize(A->stream));
  return ELL_OK;
}

extern "C" int ellpack_trace_product(const ellpack_t *A, const ellpack_t *B, double *trace_out)
{
  if (!A || !B || !trace_out || A->N != B->N) return ELL_EINVAL;
  int rc = ensure_valid(A);
  if (rc) return rc;
  rc = ensure_valid(B);
  if (rc) return rc;
  if (B->stream != A->stream) HIP_TRY(hipStreamSynchronize(B->stream));
  AllocScope scope(A->stream);
  DevMem d, part, out;
  HIP_TRY(d.alloc(sizeof(double) * A->N));
  HIP_TRY(part.alloc(sizeof(double) * ((A->N + kRedBlock - 1) / kRedBlock)));
  HIP_TRY(out.alloc(sizeof(double)));
  const bool a64 = A->prec == ELL_F64, b64 = B->prec == ELL_F64;
  if (a64 && b64)
    HIP_TRY((launch_trace_product_rows<double, double>(A->N, view<double>(A), view<double>(B), d.as<double>(),
                                                        A->stream)));
  else if (a64)
    HIP_TRY((launch_trace_product_rows<double, float>(A->N, view<double>(A), view<float>(B), d.as<double>(),
                                                       A->stream)));
  else if (b64)
    HIP_TRY((launch_trace_product_rows<float, double>(A->N, view<float>(A), view<double>(B), d.as<double>(),
                                                       A->stream)));
  else
    HIP_TRY((launch_trace_product_rows<float, float>(A->N, view<float>(A), view<float>(B), d.as<double>(),
                                                      A->stream)));
  HIP_TRY(launch_tree_sum(A->N, d.as<double>(), part.as<double>(), out.as<double>(), A->stream));
  HIP_TRY(hipMemcpyAsync(trace_out, out.p, sizeof(double), hipMemcpyDeviceToHost, A->stream));
  HIP_TRY(hipStreamSynchronize(A->stream));
  return ELL_OK;
}

// ===========================================================================
// SP2
// ===========================================================================
namespace {

// Three working matrices of one precision in ELLPACK form, capacity cap.
template <typename T>
struct WorkSet {
  DevMem nnz[3], idx[3], val[3];
  int32_t cap = 0;
  hipError_t alloc(int N, int32_t c)
  {
    cap = c;
    for (int b = 0; b < 3; ++b) {
      hipError_t e;
      if ((e = nnz[b].alloc(sizeof(int32_t) * N)) || (e = idx[b].alloc(sizeof(int32_t) * (size_t)N * c)) ||
          (e = val[b].alloc(sizeof(T) * (size_t)N * c)))
        return e;
    }
    return hipSuccess;
  }
  void release()
  {
    for (int b = 0; b < 3; ++b) {
      nnz[b].release();
      idx[b].release();
      val[b].release();
    }
    cap = 0;
  }
  EllView<T> v(int b) const { return EllView<T>{nnz[b].as<int32_t>(), idx[b].as<int32_t>(), val[b].as<T>(), cap}; }
  Rot3<T> rot() const { return Rot3<T>{{v(0), v(1), v(2)}}; }
};

// Three working matrices of one precision in span form, stride SW.
template <typename T>
struct SpanSet {
  SpanMem<T> m[3];
  int32_t SW = 0;
  hipError_t alloc(int N, int32_t sw, bool zero_values = true)
  {
    SW = sw;
    // the six interval arrays in one launch on the blocks' stream (outside an
    // allocation scope that names a stream, each with its own hipMemset)
    ZeroList z{};
    bool one = true;
    for (int b = 0; b < 3; ++b) {
      hipError_t e = m[b].alloc(N, sw, zero_values, false);
      if (e) return e;
      one = one && m[b].base.ordered() && m[b].len.ordered() && m[b].base.stream == m[0].base.stream &&
            m[b].len.stream == m[0].base.stream;
      z.p[z.count] = m[b].base.template as<int32_t>();
      z.n[z.count++] = N + kSpanPadRows;
      z.p[z.count] = m[b].len.template as<int32_t>();
      z.n[z.count++] = N + kSpanPadRows;
    }
    if (one) return launch_zero_list(z, m[0].base.stream);
    for (int b = 0; b < 3; ++b) {
      hipError_t e;
      if ((e = m[b].base.zero(sizeof(int32_t) * ((size_t)N + kSpanPadRows))) ||
          (e = m[b].len.zero(sizeof(int32_t) * ((size_t)N + kSpanPadRows))))
        return e;
    }
    return hipSuccess;
  }
  void release()
  {
    for (int b = 0; b < 3; ++b) m[b].release();
    SW = 0;
  }
  SpanView<T> v(int b) const { return m[b].v(); }
  SpanRot3<T> rot() const { return SpanRot3<T>{{v(0), v(1), v(2)}}; }
};

// Results of the initialisation kernels, read by the host with one copy and
// one synchronisation.
struct InitBlock {
  double emin, emax;            // Gershgorin bounds
  int32_t flags;                // bit 1: H holds a non-finite value
  int32_t asym;                 // bit 0: an entry above the diagonal has no equal mirror
  unsigned long long balance;   // entries above minus below the diagonal (H symmetric iff 0 and asym 0)
  // the X0 results (from wmax on: cleared when X0 is formed again)
  int32_t wmax;                 // widest row of X0
  unsigned long long total;     // entries of X0 (the extent kernel's sums: then
  unsigned long long lensum;    //   the summed row interval lengths)
  int32_t maxlen;               // longest row interval of X0
  int32_t xflags;               // bit 2: X0 stores an exact zero (never: it keeps |x| > tau >= 0)
};

// Per-iteration history, one block of arrays of max_iter entries each (device,
// and its pinned mirror): trx, trx2, eta2 (double), nnzx, nnzy (int64), maxw
// (int32), up, prec (int8).
constexpr size_t kHistBytesPerIter = 3 * 8 + 2 * 8 + 4 + 1 + 1;
constexpr size_t kHistMirrorMax = (size_t)1 << 20;  // larger histories are copied array by array

struct Solver {
  int N = 0;
  hipStream_t stream = nullptr;
  StepMem step;
  DevMem state, hist, init;
  size_t mi = 0;  // entries per history array
  DevMem glo, ghi, wmax;
  // pinned: [0] host working copy of the state, [1], [2] the poll slots; the
  // init block; the history mirror when it fits kHistMirrorMax
  PinnedMem pin;
  size_t pin_init = 0, pin_hist = 0;
  hipEvent_t polled[2] = {nullptr, nullptr};
  std::vector<hipEvent_t> events;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> marks;  // step-kernel launches when profiling
  bool profile = false;
  bool sym = false;  // H bitwise symmetric: the span iteration fixes each branch before its product
  ~Solver()
  {
    if (pin.b.p) (void)hipStreamSynchronize(stream);  // nothing queued still writes the pinned block
    pin.release();
    for (hipEvent_t e : polled)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
  }
  SP2State *host_state() const { return pin.host<SP2State>(0); }
  SP2State *host_state_dev() const { return pin.dev<SP2State>(0); }
  InitBlock *init_host() const { return pin.host<InitBlock>(pin_init); }
  InitBlock *init_dev() const { return init.as<InitBlock>(); }
  static SP2Hist hist_view(char *b, size_t mi)
  {
    return SP2Hist{reinterpret_cast<double *>(b),           reinterpret_cast<double *>(b + 8 * mi),
                   reinterpret_cast<double *>(b + 16 * mi), reinterpret_cast<int8_t *>(b + 44 * mi),
                   reinterpret_cast<int8_t *>(b + 45 * mi), reinterpret_cast<int32_t *>(b + 40 * mi),
                   reinterpret_cast<int64_t *>(b + 24 * mi), reinterpret_cast<int64_t *>(b + 32 * mi)};
  }
  SP2Hist hist_dev() const { return hist_view(hist.as<char>(), mi); }
  hipError_t mark(hipEvent_t *e)
  {
    hipError_t r = hipEventCreate(e);
    if (r == hipSuccess) events.push_back(*e);
    if (r == hipSuccess) r = hipEventRecord(*e, stream);
    return r;
  }
};

// Pipelines: the step kernel, then the reductions and the decision.
enum Pipe { PIPE_SPAN = 0, PIPE_ELL = 1 };

template <typename T>
int launch_iteration(Solver &S, Pipe pipe, const SpanSet<T> &Sp, const WorkSet<T> &W, T tau, SP2Cfg cfg,
                     SP2State *publish, bool *published)
{
  hipEvent_t a = nullptr, b = nullptr;
  if (S.profile) HIP_TRY(S.mark(&a));
  SP2State *st = S.state.as<SP2State>();
  StepScratch sc = S.step.s;
  *published = false;
  if (pipe == PIPE_SPAN && S.sym && x2_band16_fits(S.N, Sp.SW, (int)sizeof(T))) {
    // product of the branch fixed beforehand, writing that iterate only; then
    // the rest of the reduction, the decision and the next branch
    cfg.span = 1;
    HIP_TRY(launch_x2_sym_step<T>(S.N, Sp.rot(), st, tau, sc, cfg, S.hist_dev(), publish, S.stream));
    if (S.profile) {
      HIP_TRY(S.mark(&b));
      S.marks.emplace_back(a, b);
    }
    *published = publish != nullptr;
    return ELL_OK;
  }
  if (pipe == PIPE_SPAN && x2_band16_fits(S.N, Sp.SW, (int)sizeof(T))) {
    // product with 64-row partials, then the rest of the reduction and the decision
    cfg.span = 1;
    HIP_TRY(launch_x2_band16_part<T>(S.N, Sp.rot(), st, tau, sc, S.stream));
    if (S.profile) {
      HIP_TRY(S.mark(&b));
      S.marks.emplace_back(a, b);
    }
    HIP_TRY(launch_step_final64(st, cfg, S.hist_dev(), sc, publish, S.stream));
    *published = publish != nullptr;
    return ELL_OK;
  }
  if (pipe == PIPE_SPAN) {
    cfg.span = 1;
    HIP_TRY(launch_x2_band<T>(S.N, Sp.rot(), W.rot(), st, true, false, tau, sc, sc.flags, S.stream));
  } else {
    cfg.span = 0;
    sc = ell_scratch(sc);
    HIP_TRY(launch_x2_step<T>(S.N, W.rot(), st, true, tau, sc, S.stream));
  }
  if (S.profile) {
    HIP_TRY(S.mark(&b));
    S.marks.emplace_back(a, b);
  }
  HIP_TRY(launch_reduce(S.N, st, sc, S.stream));
  HIP_TRY(launch_decide(st, cfg, S.hist_dev(), sc, S.stream));
  return ELL_OK;
}

int check_params(const sp2_params_t *p)
{
  if (!p) return ELL_EINVAL;
  if (bad_tau(p->tau) || !(p->idem_target >= 0.0) || !std::isfinite(p->idem_target)) return ELL_EINVAL;
  if (p->max_iter < 1 || p->fp64_tail_steps < 0 || p->poll_every < 0) return ELL_EINVAL;
  if (p->precision != SP2_F64 && p->precision != SP2_MIXED) return ELL_EINVAL;
  if (p->precision == SP2_MIXED && (bad_tau(p->tau_fp32) || !(p->switch_eta >= 0.0))) return ELL_EINVAL;
  if (!std::isfinite(p->n_occ)) return ELL_EINVAL;
  return ELL_OK;
}

// Reallocate an owned D to capacity M (contents discarded).
int regrow_owned(ellpack *D, int32_t M)
{
  int32_t *idx = nullptr;
  double *val = nullptr;
  HIP_TRY(hipMalloc(&idx, sizeof(int32_t) * (size_t)D->N * M));
  hipError_t e = hipMalloc(&val, sizeof(double) * (size_t)D->N * M);
  if (e != hipSuccess) {
    (void)hipFree(idx);
    return device_error(e, "sp2_solve: result allocation");
  }
  (void)hipFree(D->idx);
  (void)hipFree(D->val);
  D->idx = idx;
  D->val = val;
  D->M = M;
  return ELL_OK;
}

// The final X into D (ELLPACK, FP64), reallocating an owned D when too narrow.
template <typename T>
int deliver(Solver &S, Pipe pipe, const SpanSet<T> &Sp, const WorkSet<T> &W, int cur, ellpack *D,
            int32_t *final_width)
{
  for (int attempt = 0; attempt < 2; ++attempt) {
    HIP_TRY(hipMemsetAsync(S.wmax.p, 0, sizeof(int32_t), S.stream));
    if (pipe == PIPE_SPAN) {
      HIP_TRY((launch_span_to_ell<T, double>(S.N, Sp.v(cur), view<double>(D), S.wmax.as<int32_t>(), S.stream)));
    } else {
      std::vector<int32_t> hn(S.N);
      HIP_TRY(hipMemcpyAsync(hn.data(), W.nnz[cur].p, sizeof(int32_t) * S.N, hipMemcpyDeviceToHost, S.stream));
      HIP_TRY(hipStreamSynchronize(S.stream));
      int32_t w = 0;
      for (int32_t v : hn) w = std::max(w, v);
      HIP_TRY(hipMemcpyAsync(S.wmax.p, &w, sizeof(w), hipMemcpyHostToDevice, S.stream));
      if (w <= D->M) HIP_TRY((launch_copy<T, double>(S.N, W.v(cur), view<double>(D), S.stream)));
    }
    int32_t width = 0;
    HIP_TRY(hipMemcpyAsync(&width, S.wmax.p, sizeof(width), hipMemcpyDeviceToHost, S.stream));
    HIP_TRY(hipStreamSynchronize(S.stream));
    *final_width = width;
    if (width <= D->M) {
      D->validated = true;
      return ELL_OK;
    }
    if (!D->owned) return ELL_EOVERFLOW;
    int rc = regrow_owned(D, std::max(roundup32(width), 32));
    if (rc) return rc;
  }
  return ELL_EOVERFLOW;
}

}  // namespace

extern "C" int sp2_solve(const ellpack_t *H, ellpack_t *D, const sp2_params_t *p, sp2_report_t *r)
{
  if (!H || !D || H == D || H->prec != ELL_F64 || D->prec != ELL_F64 || H->N != D->N) return ELL_EINVAL;
  if (H->val == D->val) return ELL_EINVAL;
  int rc = check_params(p);
  if (rc) return rc;
  if (r) {
    r->status = 0;
    r->iterations = r->fp32_iterations = r->final_M = 0;
    r->eta = r->trace_x = r->emin = r->emax = r->seconds = 0.0;
    r->x2_seconds = 0.0;
    r->x2_bytes = 0;
    r->x2_launches = 0;
    r->batch_k = r->batch_kernel = 0;
  }
  rc = ensure_valid(H);
  if (rc) return rc;

  const int N = H->N;
  const bool mixed = p->precision == SP2_MIXED;
  const int poll = p->poll_every > 0 ? p->poll_every : 4;
  AllocScope scope(D->stream);
  Solver S;
  S.N = N;
  S.stream = D->stream;
  S.profile = p->profile != 0;
  hipStream_t st = S.stream;
  HIP_TRY(S.step.alloc(N));
  HIP_TRY(S.state.alloc(sizeof(SP2State)));
  S.mi = (size_t)p->max_iter;
  HIP_TRY(S.hist.alloc(kHistBytesPerIter * S.mi));
  HIP_TRY(S.init.alloc(sizeof(InitBlock)));
  const int gb = gersh_blocks(N);  // Gershgorin partials, one per workgroup
  HIP_TRY(S.glo.alloc(sizeof(double) * gb));
  HIP_TRY(S.ghi.alloc(sizeof(double) * gb));
  HIP_TRY(S.wmax.alloc(sizeof(int32_t)));
  const size_t hist_bytes = kHistBytesPerIter * S.mi;
  S.pin_init = 3 * sizeof(SP2State);
  S.pin_hist = (S.pin_init + sizeof(InitBlock) + 63) / 64 * 64;
  HIP_TRY(S.pin.alloc(S.pin_hist + (hist_bytes <= kHistMirrorMax ? hist_bytes : 0)));
  for (hipEvent_t &e : S.polled) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));

  hipEvent_t t0, t1;
  HIP_TRY(S.mark(&t0));

  // Init: Gershgorin bounds, X0 (its kernel reads the bounds on the device) and
  // X0's row intervals, then one synchronisation for all their results.
  // Degenerate or non-finite spectra are reported after it; the kernels queued
  // behind the bounds stay in bounds whatever values they read.
  int32_t cap = roundup32(std::min<int64_t>((int64_t)H->M + 1, N));
  cap = std::max(cap, std::min(roundup32(D->M), roundup32(N)));
  cap = std::min(std::max(cap, 32), kMaxCap);
  WorkSet<float> W32;
  WorkSet<double> W64;
  SpanSet<float> S32;
  SpanSet<double> S64;
  InitBlock *ib = S.init_dev();
  InitBlock &hi = *S.init_host();
  HIP_TRY(hipMemsetAsync(ib, 0, sizeof(InitBlock), st));
  HIP_TRY(launch_gershgorin(N, view<double>(H), S.glo.as<double>(), S.ghi.as<double>(), &ib->emin, &ib->flags, st));
  HIP_TRY(launch_check_symmetric(N, view<double>(H), &ib->asym, &ib->balance, st));
  bool first = true;
  for (;;) {
    if (!first) {  // X0 again, wider: clear the X0 results
      HIP_TRY(hipMemsetAsync(&ib->wmax, 0, sizeof(InitBlock) - offsetof(InitBlock, wmax), st));
    }
    if (mixed) {
      HIP_TRY(W32.alloc(N, cap));
      HIP_TRY(launch_x0<float>(N, view<double>(H), W32.v(0), &ib->emin, (float)p->tau_fp32, &ib->wmax, nullptr,
                               st));
      HIP_TRY(launch_ell_extent<float>(N, W32.v(0), nullptr, nullptr, &ib->maxlen, &ib->total, st));
    } else {
      HIP_TRY(W64.alloc(N, cap));
      HIP_TRY(launch_x0<double>(N, view<double>(H), W64.v(0), &ib->emin, p->tau, &ib->wmax, nullptr, st));
      HIP_TRY(launch_ell_extent<double>(N, W64.v(0), nullptr, nullptr, &ib->maxlen, &ib->total, st));
    }
    HIP_TRY(hipMemcpyAsync(&hi, ib, sizeof(InitBlock), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (first) {
      if (hi.flags & 2) return ELL_ENONFINITE;
      if (r) {
        r->emin = hi.emin;
        r->emax = hi.emax;
      }
      if (!(hi.emax > hi.emin)) return ELL_EDEGENERATE;
      if (!(p->n_occ > 0.0 && p->n_occ < (double)N)) return ELL_EDEGENERATE;
      first = false;
    }
    if (hi.wmax <= cap) break;
    cap = roundup32(hi.wmax);
    if (cap > kMaxCap) return ELL_EOVERFLOW;
  }
  const unsigned long long nnz0 = hi.total;

  // Span pipeline when X0's rows are intervals short enough for it.
  Pipe pipe = PIPE_ELL;
  {
    const int32_t maxlen = hi.maxlen;
    const bool zeros = (hi.xflags & 4) != 0;
    // a bitwise symmetric H gives bitwise symmetric iterates: their rows are
    // read through the symmetry, in runs of kSymAlign columns
    S.sym = (hi.asym & 1) == 0 && hi.balance == 0;
    const int32_t pad = S.sym ? 2 * (kSymAlign - 1) : 0;
    const int32_t sw = std::min(std::max(256, roundup64(maxlen + pad)), std::max(64, roundup64(N)));
    // (X0's fill of its intervals does not decide here: the iterates fill them)
    if (!zeros && maxlen <= kMaxCap) {
      const int align = S.sym ? kSymAlign : 1;
      // (the symmetric iteration reads nothing outside the rows' intervals)
      const bool zero = !(S.sym && x2_band16_fits(N, sw, mixed ? (int)sizeof(float) : (int)sizeof(double)));
      if (mixed) {
        HIP_TRY(S32.alloc(N, sw, zero));
        HIP_TRY(launch_ell_to_span<float>(N, W32.v(0), S32.v(0), st, align));
      } else {
        HIP_TRY(S64.alloc(N, sw, zero));
        HIP_TRY(launch_ell_to_span<double>(N, W64.v(0), S64.v(0), st, align));
      }
      pipe = PIPE_SPAN;
    }
  }

  SP2State &hs = *S.host_state();
  std::memset(&hs, 0, sizeof(hs));
  hs.cur = 0;
  hs.status = ST_RUNNING;
  hs.phase32 = mixed ? 1 : 0;
  hs.cap = cap;
  hs.sw = mixed ? S32.SW : S64.SW;
  hs.nnz_cur = (int64_t)nnz0;
  hs.once = p->prune_once ? 1 : 0;
  HIP_TRY(hipMemcpyAsync(S.state.p, &hs, sizeof(hs), hipMemcpyHostToDevice, st));

  SP2Cfg cfg{};
  cfg.n_occ = p->n_occ;
  cfg.target2 = p->idem_target * p->idem_target;
  cfg.switch2 = p->switch_eta * p->switch_eta;
  cfg.max_iter = p->max_iter;
  cfg.tail = p->fp64_tail_steps;
  cfg.stall = p->stall_stop ? 1 : 0;
  cfg.mixed = mixed ? 1 : 0;

  // The symmetric iteration needs the branch of the first product of the
  // current X before it: from the chains of squares of X's rows.
  auto seed = [&]() -> int {
    if (pipe != PIPE_SPAN || !S.sym) return ELL_OK;
    SP2State *dst = S.state.as<SP2State>();
    if (hs.phase32) {
      if (x2_band16_fits(N, S32.SW, (int)sizeof(float)))
        HIP_TRY(launch_sym_seed<float>(N, S32.rot(), dst, cfg, S.step.s, st));
    } else {
      if (x2_band16_fits(N, S64.SW, (int)sizeof(double)))
        HIP_TRY(launch_sym_seed<double>(N, S64.rot(), dst, cfg, S.step.s, st));
    }
    return ELL_OK;
  };
  if ((rc = seed())) return rc;

  auto restart = [&]() -> int {
    hs.stop = 0;
    hs.status = ST_RUNNING;
    HIP_TRY(hipMemcpyAsync(S.state.p, &hs, sizeof(hs), hipMemcpyHostToDevice, st));
    return ELL_OK;
  };

  // A batch is `poll` iterations followed by a copy of the device state into a
  // pinned slot (written by the batch's last decision kernel itself when the
  // span form runs on the matrix cores).  The next batch is queued before the host waits for the
  // current one, so the device never idles while the host reads the state; if
  // the current batch stopped, every kernel of the next one returns at once.
  SP2State *slot = S.host_state() + 1;
  SP2State *slot_dev = S.host_state_dev() + 1;
  struct Queued {
    size_t m0 = 0, m1 = 0;  // its step-kernel marks (profiling)
    int k = 0;              // its poll slot
  };
  auto enqueue = [&](int k, Queued &b) -> int {
    b.k = k;
    b.m0 = S.marks.size();
    bool published = false;
    for (int q = 0; q < poll; ++q) {
      SP2State *pub = q == poll - 1 ? slot_dev + k : nullptr;
      const int e = hs.phase32 ? launch_iteration<float>(S, pipe, S32, W32, (float)p->tau_fp32, cfg, pub, &published)
                               : launch_iteration<double>(S, pipe, S64, W64, p->tau, cfg, pub, &published);
      if (e) return e;
    }
    b.m1 = S.marks.size();
    if (!published) HIP_TRY(hipMemcpyAsync(&slot[k], S.state.p, sizeof(SP2State), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(S.polled[k], st));
    return ELL_OK;
  };

  int status = ST_RUNNING;
  // every batch advances the iteration count or changes capacity, precision or
  // pipeline (each a bounded number of times), so this bounds the loop even if
  // the device control misbehaved
  const int64_t max_batches = (int64_t)p->max_iter + 64;
  bool fresh = true;
  Queued cur, nxt;
  for (int64_t batch = 0;; ++batch) {
    if (batch > max_batches) {
      g_last_error = "sp2_solve: device control block did not reach a stop";
      return ELL_EDEVICE;
    }
    if (fresh) {
      if ((rc = enqueue(0, cur))) return rc;
      fresh = false;
    }
    const int iter_before = hs.iter;
    // Near the end -- in the FP64 phase, the last norm squared, squared once
    // per product (SP2 converges about quadratically), falls below the target
    // within the batch waited for -- nothing is queued behind that batch: its
    // launches would only return at once after the stop.  (A wrong guess costs
    // the host's reading of the state between two batches; the results are the
    // same either way.)
    bool ahead = true;
    if (!hs.phase32 && hs.iter > 0 && hs.eta2 > 0.0) {
      double e = hs.eta2;
      for (int j = 0; j < poll && ahead; ++j) {
        e = e * e;
        ahead = !(e < cfg.target2);
      }
    }
    if (ahead) {
      if ((rc = enqueue(1 - cur.k, nxt))) return rc;
    } else {
      nxt.m0 = nxt.m1 = S.marks.size();  // (nothing queued)
    }
    HIP_TRY(hipEventSynchronize(S.polled[cur.k]));
    hs = slot[cur.k];
    if (S.profile) {
      // step kernels launched after the stop returned at once: drop them
      const bool redo = hs.stop && (hs.status == ELL_EOVERFLOW || hs.status == ST_FALLBACK);
      const int worked = hs.iter - iter_before + (redo ? 1 : 0);
      for (size_t q = cur.m0; q < cur.m1; ++q)
        if ((int)(q - cur.m0) >= worked) S.marks[q].first = nullptr;
    }
    if (!hs.stop) {
      if (ahead) cur = nxt;
      else fresh = true;  // the guess was early: queue the next batch now
      continue;
    }
    // the batch queued behind it (if any) saw the stop flag: let it drain
    HIP_TRY(hipStreamSynchronize(st));
    for (size_t q = nxt.m0; q < nxt.m1; ++q) S.marks[q].first = nullptr;
    fresh = true;
    if (hs.status == ELL_EOVERFLOW) {
      const int32_t need = hs.need_width;
      if (pipe == PIPE_SPAN) {
        const int32_t sw = roundup64(need);
        if (sw > kMaxCap) {
          hs.status = ST_FALLBACK;  // continue on ELLPACK rather than grow the interval stride further
        } else {
          if (hs.phase32) {
            SpanSet<float> G;
            HIP_TRY(G.alloc(N, sw));
            HIP_TRY((launch_span_copy<float, float>(N, S32.v(hs.cur), G.v(0), st)));
            HIP_TRY(hipStreamSynchronize(st));
            S32.release();
            for (int b = 0; b < 3; ++b) {
              swap_mem(S32.m[b].val, G.m[b].val);
              swap_mem(S32.m[b].base, G.m[b].base);
              swap_mem(S32.m[b].len, G.m[b].len);
              S32.m[b].SW = sw;
            }
            S32.SW = sw;
          } else {
            SpanSet<double> G;
            HIP_TRY(G.alloc(N, sw));
            HIP_TRY((launch_span_copy<double, double>(N, S64.v(hs.cur), G.v(0), st)));
            HIP_TRY(hipStreamSynchronize(st));
            S64.release();
            for (int b = 0; b < 3; ++b) {
              swap_mem(S64.m[b].val, G.m[b].val);
              swap_mem(S64.m[b].base, G.m[b].base);
              swap_mem(S64.m[b].len, G.m[b].len);
              S64.m[b].SW = sw;
            }
            S64.SW = sw;
          }
          hs.cur = 0;
          hs.sw = sw;
          if ((rc = restart())) return rc;
          continue;
        }
      } else {
        const int32_t newcap = roundup32(need);
        if (newcap > kMaxCap) {
          status = ELL_EOVERFLOW;
          break;
        }
        if (hs.phase32) {
          WorkSet<float> G;
          HIP_TRY(G.alloc(N, newcap));
          HIP_TRY((launch_copy<float, float>(N, W32.v(hs.cur), G.v(0), st)));
          HIP_TRY(hipStreamSynchronize(st));
          W32.release();
          for (int b = 0; b < 3; ++b) {
            swap_mem(W32.nnz[b], G.nnz[b]);
            swap_mem(W32.idx[b], G.idx[b]);
            swap_mem(W32.val[b], G.val[b]);
          }
          W32.cap = newcap;
        } else {
          WorkSet<double> G;
          HIP_TRY(G.alloc(N, newcap));
          HIP_TRY((launch_copy<double, double>(N, W64.v(hs.cur), G.v(0), st)));
          HIP_TRY(hipStreamSynchronize(st));
          W64.release();
          for (int b = 0; b < 3; ++b) {
            swap_mem(W64.nnz[b], G.nnz[b]);
            swap_mem(W64.idx[b], G.idx[b]);
            swap_mem(W64.val[b], G.val[b]);
          }
          W64.cap = newcap;
        }
        hs.cur = 0;
        hs.cap = newcap;
        if ((rc = restart())) return rc;
        continue;
      }
    }
    if (hs.status == ST_FALLBACK) {
      // the current X (span form) into ELLPACK working matrices of capacity SW
      const int32_t c = std::min(std::max(32, roundup32(hs.phase32 ? S32.SW : S64.SW)), kMaxCap);
      HIP_TRY(hipMemsetAsync(S.wmax.p, 0, sizeof(int32_t), st));
      if (hs.phase32) {
        HIP_TRY(W32.alloc(N, c));
        HIP_TRY((launch_span_to_ell<float, float>(N, S32.v(hs.cur), W32.v(0), S.wmax.as<int32_t>(), st)));
      } else {
        HIP_TRY(W64.alloc(N, c));
        HIP_TRY((launch_span_to_ell<double, double>(N, S64.v(hs.cur), W64.v(0), S.wmax.as<int32_t>(), st)));
      }
      int32_t w = 0;
      HIP_TRY(hipMemcpyAsync(&w, S.wmax.p, sizeof(w), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (w > c) {
        status = ELL_EOVERFLOW;
        break;
      }
      S32.release();
      S64.release();
      pipe = PIPE_ELL;
      hs.cur = 0;
      hs.cap = c;
      if ((rc = restart())) return rc;
      continue;
    }
    if (hs.status == ST_SWITCH) {
      if (pipe == PIPE_SPAN) {
        HIP_TRY(S64.alloc(N, S32.SW, !(S.sym && x2_band16_fits(N, S32.SW, (int)sizeof(double)))));
        HIP_TRY((launch_span_copy<float, double>(N, S32.v(hs.cur), S64.v(0), st)));
        HIP_TRY(hipStreamSynchronize(st));
        S32.release();
        hs.sw = S64.SW;
      } else {
        HIP_TRY(W64.alloc(N, W32.cap));
        HIP_TRY((launch_copy<float, double>(N, W32.v(hs.cur), W64.v(0), st)));
        HIP_TRY(hipStreamSynchronize(st));
        W32.release();
        hs.cap = W64.cap;
      }
      hs.cur = 0;
      hs.phase32 = 0;
      if ((rc = restart())) return rc;
      if ((rc = seed())) return rc;  // the FP64 traces of the widened X fix its first branch
      continue;
    }
    if (hs.status == ST_MISPREDICT) {  // (the report holds the history up to that product)
      g_last_error = "sp2_solve: the traces of an iterate differ from those its branch was chosen with";
      status = ELL_EDEVICE;
      break;
    }
    status = hs.status;
    break;
  }
  HIP_TRY(S.mark(&t1));

  // the history into its pinned mirror, covered by deliver's synchronisation
  const int n = hs.iter;
  const bool mirror = S.pin.b.bytes >= S.pin_hist + kHistBytesPerIter * S.mi;
  if (r && n > 0 && mirror)
    HIP_TRY(hipMemcpyAsync(S.pin.host<char>(S.pin_hist), S.hist.p, kHistBytesPerIter * S.mi, hipMemcpyDeviceToHost,
                           st));
  int32_t width = 0;
  rc = hs.phase32 ? deliver<float>(S, pipe, S32, W32, hs.cur, D, &width)
                  : deliver<double>(S, pipe, S64, W64, hs.cur, D, &width);
  const int final_status = rc ? rc : status;
  if (!r) return final_status;

  r->status = final_status;
  r->iterations = hs.iter;
  r->final_M = pipe == PIPE_SPAN ? (hs.phase32 ? S32.SW : S64.SW) : (hs.phase32 ? W32.cap : W64.cap);
  if (rc == ELL_EOVERFLOW) r->final_M = width;
  r->eta = std::sqrt(hs.eta2);
  r->trace_x = hs.trx;
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, t0, t1));
  r->seconds = ms * 1e-3;
  std::vector<double> a(n), b(n), c(n);
  std::vector<int8_t> up(n), pr(n);
  std::vector<int32_t> mw(n);
  std::vector<int64_t> nx(n), ny(n);
  if (n > 0) {
    const SP2Hist hd = S.hist_dev();
    SP2Hist h = hd;
    if (mirror) {
      HIP_TRY(hipStreamSynchronize(st));  // normally already done by deliver
      h = Solver::hist_view(S.pin.host<char>(S.pin_hist), S.mi);
    } else {
      h = SP2Hist{a.data(), b.data(), c.data(), up.data(), pr.data(), mw.data(), nx.data(), ny.data()};
      HIP_TRY(hipMemcpyAsync(a.data(), hd.trx, sizeof(double) * n, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(b.data(), hd.trx2, sizeof(double) * n, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(c.data(), hd.eta2, sizeof(double) * n, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(up.data(), hd.up, n, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(pr.data(), hd.prec, n, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(mw.data(), hd.maxw, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(nx.data(), hd.nnzx, sizeof(int64_t) * n, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(ny.data(), hd.nnzy, sizeof(int64_t) * n, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
    }
    if (mirror) {
      std::copy(h.trx, h.trx + n, a.begin());
      std::copy(h.trx2, h.trx2 + n, b.begin());
      std::copy(h.eta2, h.eta2 + n, c.begin());
      std::copy(h.up, h.up + n, up.begin());
      std::copy(h.prec, h.prec + n, pr.begin());
      std::copy(h.maxw, h.maxw + n, mw.begin());
      std::copy(h.nnzx, h.nnzx + n, nx.begin());
      std::copy(h.nnzy, h.nnzy + n, ny.begin());
    }
  }
  int f32 = 0;
  for (int q = 0; q < n; ++q) f32 += pr[q] ? 1 : 0;
  r->fp32_iterations = f32;
  for (int q = 0; q < n; ++q) {
    if (r->hist_trx) r->hist_trx[q] = a[q];
    if (r->hist_trx2) r->hist_trx2[q] = b[q];
    if (r->hist_eta2) r->hist_eta2[q] = c[q];
    if (r->hist_up) r->hist_up[q] = up[q];
    if (r->hist_prec) r->hist_prec[q] = pr[q];
    if (r->hist_maxw) r->hist_maxw[q] = mw[q];
  }
  int64_t bytes = 0;
  for (int q = 0; q < n; ++q) {
    const int64_t sv = pr[q] ? 4 : 8;
    const int64_t bq = nx[q] * (sv + 4) + 4LL * N + ny[q] * (sv + 4) + 4LL * N;
    if (r->hist_x2_bytes) r->hist_x2_bytes[q] = bq;
    bytes += bq;
  }
  r->x2_bytes = bytes;
  if (S.profile) {
    double sec = 0.0;
    int launches = 0;
    for (auto &m : S.marks) {
      if (!m.first) continue;
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, m.first, m.second));
      sec += t * 1e-3;
      if (r->hist_x2_seconds && launches < p->max_iter) r->hist_x2_seconds[launches] = t * 1e-3;
      ++launches;
    }
    r->x2_seconds = sec;
    r->x2_launches = launches;
  }
  return final_status;
}

// ===========================================================================
// batched SP2
// ===========================================================================
namespace {

struct BatchInst {
  int q = 0;                 // index in the caller's arrays
  int N = 0, r0 = 0;         // rows; first row in the stacked matrix
  int nb = 0, pb = 0;        // reduction blocks; first partial block
  int hoff = 0;              // offset of its history arrays
  bool mixed = false;
  double emin = 0, emax = 0;
  int32_t maxlen = 0;
  unsigned long long nnz0 = 0;
  int status = ST_RUNNING;   // set when the instance leaves the batch before the loop
  bool solo = false;         // finished by sp2_solve on its own (the batch cannot hold it)
};

// What the batched solve's tuner chose -- graph length and step kernel -- per
// device architecture, precision mix and size class (log2 of the stacked rows
// and of the row stride), kept for the life of the process.
struct BatchTune {
  int K = 0, kernel = 0;
};
std::mutex g_tune_mu;
std::vector<std::pair<std::string, BatchTune>> g_tune;

std::string batch_tune_key(int NT, int SW, bool any32)
{
  int dev = 0;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  auto lg = [](int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
  };
  return arch + (any32 ? "|mixed|" : "|f64|") + std::to_string(lg(NT)) + "|" + std::to_string(lg(SW));
}

bool batch_tune_get(const std::string &key, BatchTune *t)
{
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto &e : g_tune)
    if (e.first == key) {
      *t = e.second;
      return true;
    }
  return false;
}

void batch_tune_put(const std::string &key, BatchTune t)
{
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto &e : g_tune)
    if (e.first == key) {
      e.second = t;
      return;
    }
  g_tune.emplace_back(key, t);
}

struct Batch {
  hipStream_t st = nullptr;
  int n = 0, NT = 0, ngroups = 0, nblocks = 0, SW = 0;
  bool any32 = false;
  std::vector<BatchInst> in;
  SpanSet<double> A64;
  SpanSet<float> A32;
  DevMem d1, d2, e, wy, wu, ly, lu, part, partw, partn, out, outw, outn, flags;
  DevMem grp_inst, blk_inst, blk_local, inst_rows, inst_r0, ss, states, cfgs, hists, taus64, taus32;
  DevMem h_trx, h_trx2, h_eta2, h_up, h_prec, h_maxw, h_nnzx, h_nnzy;
  SP2State *hs = nullptr;    // pinned host mirror of the states
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_iters = 0;
  int kernel = 0;            // step kernel: 0 matrix cores, 1 register-tiled VALU (same results)
  bool sym = false;          // every instance's H is bitwise symmetric (so is each iterate)
  int graph_kernel = 0;      // the kernel the graph was captured with
  ~Batch()
  {
    drop_graph();
    if (hs) (void)hipHostFree(hs);
    if (st) (void)hipStreamDestroy(st);
  }
  void drop_graph()
  {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    graph_iters = 0;
  }
  StepScratch global_scratch() const
  {
    StepScratch t{};
    t.d1 = d1.as<double>();
    t.d2 = d2.as<double>();
    t.e = e.as<double>();
    t.wy = wy.as<int32_t>();
    t.wu = wu.as<int32_t>();
    t.ly = ly.as<int32_t>();
    t.lu = lu.as<int32_t>();
    return t;
  }
  template <typename T>
  SpanView<T> rows(const SpanSet<T> &A, int b, const BatchInst &m) const
  {
    SpanView<T> v = A.v(b);
    v.val += (size_t)m.r0 * v.SW;
    v.base += m.r0;
    v.len += m.r0;
    return v;
  }
  // one SP2 iteration of every running instance, as recorded into the graph
  int record_iteration()
  {
    const SP2State *stp = states.as<SP2State>();
    if (any32)
      HIP_TRY(launch_x2_band_batch<float>(ngroups, A32.rot(), grp_inst.as<int32_t>(), inst_r0.as<int32_t>(),
                                          inst_rows.as<int32_t>(), stp, 1, taus32.as<float>(),
                                          ss.as<StepScratch>(), flags.as<int32_t>(), st, kernel == 0, sym));
    HIP_TRY(launch_x2_band_batch<double>(ngroups, A64.rot(), grp_inst.as<int32_t>(), inst_r0.as<int32_t>(),
                                         inst_rows.as<int32_t>(), stp, 0, taus64.as<double>(), ss.as<StepScratch>(),
                                         flags.as<int32_t>(), st, kernel == 0, sym));
    HIP_TRY(launch_reduce_batch(nblocks, blk_inst.as<int32_t>(), blk_local.as<int32_t>(), inst_rows.as<int32_t>(),
                                ss.as<StepScratch>(), stp, st));
    HIP_TRY(launch_decide_batch(n, states.as<SP2State>(), cfgs.as<SP2Cfg>(), hists.as<SP2Hist>(),
                                ss.as<StepScratch>(), st));
    return ELL_OK;
  }
  // a graph of `iters` iterations (kernel nodes only)
  int capture(int iters)
  {
    drop_graph();
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int rc = ELL_OK;
    for (int q = 0; q < iters && rc == ELL_OK; ++q) rc = record_iteration();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    HIP_TRY(e);
    graph = g;
    HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    graph_iters = iters;
    graph_kernel = kernel;
    return ELL_OK;
  }
};

// Reallocate the stacked matrices with stride sw; every instance's current
// matrix moves to buffer 0 (its values do not depend on the stride).
int batch_regrow(Batch &B, int32_t sw)
{
  SpanSet<double> G64;
  SpanSet<float> G32;
  HIP_TRY(G64.alloc(B.NT, sw));
  if (B.any32) HIP_TRY(G32.alloc(B.NT, sw));
  for (int m = 0; m < B.n; ++m) {
    const BatchInst &I = B.in[m];
    if (I.solo) continue;
    const SP2State &h = B.hs[m];
    if (h.phase32)
      HIP_TRY((launch_span_copy<float, float>(I.N, B.rows(B.A32, h.cur, I), B.rows(G32, 0, I), B.st)));
    else
      HIP_TRY((launch_span_copy<double, double>(I.N, B.rows(B.A64, h.cur, I), B.rows(G64, 0, I), B.st)));
    B.hs[m].cur = 0;
    B.hs[m].sw = sw;
  }
  HIP_TRY(hipStreamSynchronize(B.st));
  for (int b = 0; b < 3; ++b) {
    swap_mem(B.A64.m[b].val, G64.m[b].val);
    swap_mem(B.A64.m[b].base, G64.m[b].base);
    swap_mem(B.A64.m[b].len, G64.m[b].len);
    B.A64.m[b].SW = sw;
    if (B.any32) {
      swap_mem(B.A32.m[b].val, G32.m[b].val);
      swap_mem(B.A32.m[b].base, G32.m[b].base);
      swap_mem(B.A32.m[b].len, G32.m[b].len);
      B.A32.m[b].SW = sw;
    }
  }
  B.A64.SW = sw;
  if (B.any32) B.A32.SW = sw;
  B.SW = sw;
  B.drop_graph();
  return ELL_OK;
}

// The result of instance m into D (FP64 ELLPACK, local columns).
template <typename T>
int batch_deliver(Batch &B, const SpanSet<T> &A, int m, ellpack *D, DevMem &wmax, int32_t *final_width)
{
  const BatchInst &I = B.in[m];
  for (int attempt = 0; attempt < 2; ++attempt) {
    HIP_TRY(hipMemsetAsync(wmax.p, 0, sizeof(int32_t), B.st));
    HIP_TRY((launch_span_to_ell<T, double>(I.N, B.rows(A, B.hs[m].cur, I), view<double>(D), wmax.as<int32_t>(),
                                           B.st)));
    int32_t width = 0;
    HIP_TRY(hipMemcpyAsync(&width, wmax.p, sizeof(width), hipMemcpyDeviceToHost, B.st));
    HIP_TRY(hipStreamSynchronize(B.st));
    *final_width = width;
    if (width <= D->M) {
      D->validated = true;
      return ELL_OK;
    }
    if (!D->owned) return ELL_EOVERFLOW;
    int rc = regrow_owned(D, std::max(roundup32(width), 32));
    if (rc) return rc;
  }
  return ELL_EOVERFLOW;
}

}  // namespace

extern "C" int sp2_solve_batched(int32_t n, const ellpack_t *const *H, ellpack_t *const *D, const sp2_params_t *p,
                                 sp2_report_t *r)
{
  if (n < 0 || (n > 0 && (!H || !D || !p))) return ELL_EINVAL;
  for (int32_t q = 0; q < n; ++q) {
    const ellpack *h = H[q], *d = D[q];
    if (!h || !d || h == d || h->prec != ELL_F64 || d->prec != ELL_F64 || h->N != d->N || h->val == d->val)
      return ELL_EINVAL;
    for (int32_t o = 0; o < q; ++o)
      if (D[o] == d || D[o]->val == d->val || H[o] == d) return ELL_EINVAL;
    int rc = check_params(&p[q]);
    if (rc) return rc;
  }
  for (int32_t q = 0; q < n; ++q)
    if (r) {
      r[q].status = 0;
      r[q].iterations = r[q].fp32_iterations = r[q].final_M = 0;
      r[q].eta = r[q].trace_x = r[q].emin = r[q].emax = r[q].seconds = r[q].x2_seconds = 0.0;
      r[q].x2_bytes = 0;
      r[q].x2_launches = 0;
      r[q].batch_k = r[q].batch_kernel = 0;
    }
  if (n == 0) return ELL_OK;
  for (int32_t q = 0; q < n; ++q) {
    int rc = ensure_valid(H[q]);
    if (rc) return rc;
  }
  // the callers' streams first, then a private stream for the batch
  for (int32_t q = 0; q < n; ++q) {
    HIP_TRY(hipStreamSynchronize(H[q]->stream));
    HIP_TRY(hipStreamSynchronize(D[q]->stream));
  }
  Batch B;
  HIP_TRY(hipStreamCreateWithFlags(&B.st, hipStreamNonBlocking));
  hipStream_t st = B.st;
  // the batch's buffers are plain allocations whose fills are queued on st,
  // ahead of the kernels that write them
  AllocScope fills_on_st(st, false);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  struct Ev {
    hipEvent_t &a, &b;
    ~Ev()
    {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev{t0, t1};
  HIP_TRY(hipEventCreate(&t0));
  HIP_TRY(hipEventCreate(&t1));
  HIP_TRY(hipEventRecord(t0, st));

  // ---- Gershgorin bounds of every instance (one launch, one synchronisation) ----
  std::vector<InitInst> gin_h(n);
  std::vector<int32_t> gw(n);
  int gwork = 0;
  for (int32_t q = 0; q < n; ++q) {
    gin_h[q] = InitInst{};
    gin_h[q].H = view<double>(H[q]);
    gin_h[q].N = H[q]->N;
    gin_h[q].w0 = gw[q] = gwork;
    gin_h[q].nw = gersh_blocks(H[q]->N);
    gwork += gin_h[q].nw;
  }
  DevMem gin, gws, glo, ghi, gout, gflags;
  HIP_TRY(gin.alloc(sizeof(InitInst) * n));
  HIP_TRY(gws.alloc(sizeof(int32_t) * n));
  HIP_TRY(glo.alloc(sizeof(double) * gwork));
  HIP_TRY(ghi.alloc(sizeof(double) * gwork));
  HIP_TRY(gout.alloc(sizeof(double) * 2 * n));
  HIP_TRY(gflags.alloc(sizeof(int32_t) * n));
  HIP_TRY(hipMemcpyAsync(gin.p, gin_h.data(), sizeof(InitInst) * n, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(gws.p, gw.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(gflags.p, 0, sizeof(int32_t) * n, st));
  HIP_TRY(launch_gershgorin_multi(gin.as<InitInst>(), gws.as<int32_t>(), n, gwork, glo.as<double>(),
                                  ghi.as<double>(), gout.as<double>(), gflags.as<int32_t>(), st));
  std::vector<double> ee(2 * (size_t)n);
  std::vector<int32_t> gf(n);
  HIP_TRY(hipMemcpyAsync(ee.data(), gout.p, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(gf.data(), gflags.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));

  // ---- layout: instances that can start, widest first, each at a multiple of kBatchAlign rows ----
  std::vector<int> order;
  std::vector<int> early(n, ST_RUNNING);
  for (int32_t q = 0; q < n; ++q) {
    const double lo = ee[2 * q], hi = ee[2 * q + 1];
    if (r) {
      r[q].emin = lo;
      r[q].emax = hi;
    }
    if (gf[q] & 2) early[q] = ELL_ENONFINITE;
    else if (!(hi > lo) || !(p[q].n_occ > 0.0 && p[q].n_occ < (double)H[q]->N)) early[q] = ELL_EDEGENERATE;
    else order.push_back(q);
  }
  // row-width buckets: instances sorted by the widest row of H (descending), so the
  // heaviest row groups are dispatched first and the grid's tail is short
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (int64_t)H[a]->M * H[a]->N > (int64_t)H[b]->M * H[b]->N;
  });
  B.n = (int)order.size();
  int rows = 0, blocks = 0, hoff = 0;
  for (int m = 0; m < B.n; ++m) {
    BatchInst I;
    I.q = order[m];
    I.N = H[I.q]->N;
    I.r0 = rows;
    I.nb = (I.N + kRedBlock - 1) / kRedBlock;
    I.pb = blocks;
    I.hoff = hoff;
    I.mixed = p[I.q].precision == SP2_MIXED;
    I.emin = ee[2 * I.q];
    I.emax = ee[2 * I.q + 1];
    rows += (I.N + kBatchAlign - 1) / kBatchAlign * kBatchAlign;
    blocks += I.nb;
    hoff += p[I.q].max_iter;
    B.any32 = B.any32 || I.mixed;
    B.in.push_back(I);
  }
  B.NT = rows;
  B.ngroups = rows / kGroupRows;
  B.nblocks = blocks;
  int worst = ELL_OK;
  auto note = [&](int rc) {
    if (rc != ELL_OK && (worst == ELL_OK || rc < worst)) worst = rc;
  };
  for (int32_t q = 0; q < n; ++q)
    if (early[q] != ST_RUNNING) {
      note(early[q]);
      if (r) r[q].status = early[q];
    }
  if (B.n == 0) return worst;

  // ---- bitwise symmetry of every H: if all are, so is every iterate, and the
  // matrix-core step reads its A operand through the symmetry ----
  {
    // per instance: the flag word, a pad word, then the balance
    std::vector<InitInst> ci(B.n);
    std::vector<int32_t> cw(B.n);
    int cwork = 0;
    for (int m = 0; m < B.n; ++m) {
      ci[m] = InitInst{};
      ci[m].H = view<double>(H[B.in[m].q]);
      ci[m].N = B.in[m].N;
      ci[m].w0 = cw[m] = cwork;
      ci[m].nw = sym_blocks(B.in[m].N);
      cwork += ci[m].nw;
    }
    DevMem asym, cin, cws;
    HIP_TRY(asym.alloc(sizeof(int32_t) * 4 * B.n));
    HIP_TRY(cin.alloc(sizeof(InitInst) * B.n));
    HIP_TRY(cws.alloc(sizeof(int32_t) * B.n));
    HIP_TRY(hipMemcpyAsync(cin.p, ci.data(), sizeof(InitInst) * B.n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(cws.p, cw.data(), sizeof(int32_t) * B.n, hipMemcpyHostToDevice, st));
    HIP_TRY(launch_zero_words(4 * B.n, asym.as<int32_t>(), st));
    HIP_TRY(launch_check_symmetric_multi(cin.as<InitInst>(), cws.as<int32_t>(), B.n, cwork, asym.as<int32_t>(), st));
    std::vector<int32_t> fl(4 * (size_t)B.n);
    HIP_TRY(hipMemcpyAsync(fl.data(), asym.p, sizeof(int32_t) * 4 * B.n, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    B.sym = true;
    for (int m = 0; m < B.n; ++m)
      B.sym = B.sym && (fl[4 * m] & 1) == 0 && fl[4 * m + 2] == 0 && fl[4 * m + 3] == 0;
  }

  // ---- X0 of every instance in ELLPACK form (capacity grows until it fits) ----
  // One launch per precision over the packed rows.  Rows that hold no X0 of a
  // precision (other instances, the padding between instances) keep 0 entries
  // in its buffer, so that the whole-buffer launches below leave them empty.
  int32_t cap0 = 32;
  for (const BatchInst &I : B.in)
    cap0 = std::max(cap0, std::min(roundup32(std::min<int64_t>((int64_t)H[I.q]->M + 1, I.N)), kMaxCap));
  std::vector<InitInst> xi(B.n);
  std::vector<int32_t> xr(B.n);
  for (int m = 0; m < B.n; ++m) {
    const BatchInst &I = B.in[m];
    xi[m] = InitInst{};
    xi[m].H = view<double>(H[I.q]);
    xi[m].N = I.N;
    xi[m].r0 = xr[m] = I.r0;  // (ascending in m)
    xi[m].f32 = I.mixed ? 1 : 0;
    xi[m].emax = I.emax;
    xi[m].inv = 1.0 / (I.emax - I.emin);
    xi[m].tau = I.mixed ? p[I.q].tau_fp32 : p[I.q].tau;
  }
  WorkSet<double> X64;
  WorkSet<float> X32;
  DevMem xin, xrs, rowc, lens64, lens32;
  HIP_TRY(xin.alloc(sizeof(InitInst) * B.n));
  HIP_TRY(xrs.alloc(sizeof(int32_t) * B.n));
  HIP_TRY(rowc.alloc(sizeof(int32_t) * B.NT));
  HIP_TRY(lens64.alloc(sizeof(int32_t) * B.NT));
  if (B.any32) HIP_TRY(lens32.alloc(sizeof(int32_t) * B.NT));
  HIP_TRY(hipMemcpyAsync(xin.p, xi.data(), sizeof(InitInst) * B.n, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(xrs.p, xr.data(), sizeof(int32_t) * B.n, hipMemcpyHostToDevice, st));
  HIP_TRY(rowc.zero(sizeof(int32_t) * B.NT));
  std::vector<int32_t> hc(B.NT), w0(B.n);
  std::vector<unsigned long long> nz0(B.n);
  for (;;) {
    X64.release();
    X32.release();
    // one temporary slot set of each precision in use (only buffer 0 is used)
    HIP_TRY(X64.nnz[0].alloc(sizeof(int32_t) * B.NT));
    HIP_TRY(X64.idx[0].alloc(sizeof(int32_t) * (size_t)B.NT * cap0));
    HIP_TRY(X64.val[0].alloc(sizeof(double) * (size_t)B.NT * cap0));
    HIP_TRY(X64.nnz[0].zero(sizeof(int32_t) * B.NT));
    X64.cap = cap0;
    HIP_TRY(launch_x0_multi<double>(xin.as<InitInst>(), xrs.as<int32_t>(), B.n, B.NT, X64.v(0), rowc.as<int32_t>(),
                                    st));
    if (B.any32) {
      HIP_TRY(X32.nnz[0].alloc(sizeof(int32_t) * B.NT));
      HIP_TRY(X32.idx[0].alloc(sizeof(int32_t) * (size_t)B.NT * cap0));
      HIP_TRY(X32.val[0].alloc(sizeof(float) * (size_t)B.NT * cap0));
      HIP_TRY(X32.nnz[0].zero(sizeof(int32_t) * B.NT));
      X32.cap = cap0;
      HIP_TRY(launch_x0_multi<float>(xin.as<InitInst>(), xrs.as<int32_t>(), B.n, B.NT, X32.v(0), rowc.as<int32_t>(),
                                     st));
    }
    HIP_TRY(hipMemcpyAsync(hc.data(), rowc.p, sizeof(int32_t) * B.NT, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int m = 0; m < B.n; ++m) {  // widest row and entries of each X0 (before the capacity cut)
      const BatchInst &I = B.in[m];
      int32_t w = 0;
      unsigned long long t = 0;
      for (int i = 0; i < I.N; ++i) {
        w = std::max(w, hc[I.r0 + i]);
        t += (unsigned long long)hc[I.r0 + i];
      }
      w0[m] = w;
      nz0[m] = t;
    }
    int32_t wide = 0;
    for (int32_t w : w0) wide = std::max(wide, w);
    if (wide <= cap0) break;
    if (roundup32(wide) > kMaxCap) {
      // an X0 row wider than any capacity: those instances run on their own
      for (int m = 0; m < B.n; ++m)
        if (w0[m] > kMaxCap) B.in[m].solo = true;
      bool any = false;
      for (int m = 0; m < B.n; ++m) {
        if (!B.in[m].solo) any = true;
      }
      if (!any) break;
      int32_t c = cap0;
      for (int m = 0; m < B.n; ++m)
        if (!B.in[m].solo) c = std::max(c, roundup32(w0[m]));
      if (c == cap0) break;
      cap0 = c;
      continue;
    }
    cap0 = roundup32(wide);
  }
  // ---- interval extents (one launch per precision over the packed rows);
  // instances the span form cannot hold run on their own ----
  // (an X0 keeps |x| > tau >= 0: no exact zero, which the span form could not hold)
  HIP_TRY(launch_ell_extent<double>(B.NT, X64.v(0), lens64.as<int32_t>(), nullptr, nullptr, nullptr, st));
  if (B.any32) HIP_TRY(launch_ell_extent<float>(B.NT, X32.v(0), lens32.as<int32_t>(), nullptr, nullptr, nullptr, st));
  std::vector<int32_t> hl64(B.NT), hl32(B.any32 ? B.NT : 0);
  HIP_TRY(hipMemcpyAsync(hl64.data(), lens64.p, sizeof(int32_t) * B.NT, hipMemcpyDeviceToHost, st));
  if (B.any32) HIP_TRY(hipMemcpyAsync(hl32.data(), lens32.p, sizeof(int32_t) * B.NT, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  int32_t sw = 64;
  for (int m = 0; m < B.n; ++m) {
    BatchInst &I = B.in[m];
    if (I.solo) continue;
    const std::vector<int32_t> &hl = I.mixed ? hl32 : hl64;
    for (int i = 0; i < I.N; ++i) I.maxlen = std::max(I.maxlen, hl[I.r0 + i]);
    if (I.maxlen > kMaxCap) {
      I.solo = true;
      continue;
    }
    sw = std::max(sw, std::min(std::max(256, roundup64(I.maxlen)), std::max(64, roundup64(I.N))));
    I.nnz0 = nz0[m];
  }
  B.SW = sw;
  HIP_TRY(B.A64.alloc(B.NT, sw));
  if (B.any32) HIP_TRY(B.A32.alloc(B.NT, sw));
  // rows of the instances that run on their own stay empty in span form (their
  // intervals may not fit the span width)
  for (int m = 0; m < B.n; ++m) {
    const BatchInst &I = B.in[m];
    if (!I.solo) continue;
    int32_t *nz = I.mixed ? X32.nnz[0].as<int32_t>() : X64.nnz[0].as<int32_t>();
    HIP_TRY(hipMemsetAsync(nz + I.r0, 0, sizeof(int32_t) * I.N, st));
  }
  HIP_TRY(launch_ell_to_span<double>(B.NT, X64.v(0), B.A64.v(0), st));
  if (B.any32) HIP_TRY(launch_ell_to_span<float>(B.NT, X32.v(0), B.A32.v(0), st));
  HIP_TRY(hipStreamSynchronize(st));
  X64.release();
  X32.release();

  // ---- per-instance scratch, state, configuration and history ----
  const size_t NT = (size_t)B.NT;
  HIP_TRY(B.d1.alloc(sizeof(double) * NT));
  HIP_TRY(B.d2.alloc(sizeof(double) * NT));
  HIP_TRY(B.e.alloc(sizeof(double) * NT));
  HIP_TRY(B.wy.alloc(sizeof(int32_t) * NT));
  HIP_TRY(B.wu.alloc(sizeof(int32_t) * NT));
  HIP_TRY(B.ly.alloc(sizeof(int32_t) * NT));
  HIP_TRY(B.lu.alloc(sizeof(int32_t) * NT));
  HIP_TRY(B.part.alloc(sizeof(double) * 3 * B.nblocks));
  HIP_TRY(B.partw.alloc(sizeof(int32_t) * 4 * B.nblocks));
  HIP_TRY(B.partn.alloc(sizeof(int64_t) * 2 * B.nblocks));
  HIP_TRY(B.out.alloc(sizeof(double) * 3 * B.n));
  HIP_TRY(B.outw.alloc(sizeof(int32_t) * 4 * B.n));
  HIP_TRY(B.outn.alloc(sizeof(int64_t) * 2 * B.n));
  HIP_TRY(B.flags.alloc(sizeof(int32_t) * B.n));
  HIP_TRY(hipMemsetAsync(B.flags.p, 0, sizeof(int32_t) * B.n, st));
  const size_t HT = (size_t)std::max(hoff, 1);
  HIP_TRY(B.h_trx.alloc(sizeof(double) * HT));
  HIP_TRY(B.h_trx2.alloc(sizeof(double) * HT));
  HIP_TRY(B.h_eta2.alloc(sizeof(double) * HT));
  HIP_TRY(B.h_up.alloc(HT));
  HIP_TRY(B.h_prec.alloc(HT));
  HIP_TRY(B.h_maxw.alloc(sizeof(int32_t) * HT));
  HIP_TRY(B.h_nnzx.alloc(sizeof(int64_t) * HT));
  HIP_TRY(B.h_nnzy.alloc(sizeof(int64_t) * HT));
  std::vector<int32_t> gi(B.ngroups), bi(B.nblocks), bl(B.nblocks), ir(B.n), i0(B.n);
  std::vector<StepScratch> vs(B.n);
  std::vector<SP2Cfg> vc(B.n);
  std::vector<SP2Hist> vh(B.n);
  std::vector<double> t64(B.n);
  std::vector<float> t32(B.n);
  HIP_TRY(hipHostMalloc((void **)&B.hs, sizeof(SP2State) * B.n, hipHostMallocDefault));
  const StepScratch gs = B.global_scratch();
  for (int m = 0; m < B.n; ++m) {
    const BatchInst &I = B.in[m];
    const sp2_params_t &P = p[I.q];
    const int rows_m = (I.N + kBatchAlign - 1) / kBatchAlign * kBatchAlign;
    for (int g = I.r0 / kGroupRows; g < (I.r0 + rows_m) / kGroupRows; ++g) gi[g] = m;
    for (int b = 0; b < I.nb; ++b) {
      bi[I.pb + b] = m;
      bl[I.pb + b] = b;
    }
    ir[m] = I.N;
    i0[m] = I.r0;
    StepScratch &s = vs[m];
    s.d1 = gs.d1 + I.r0;
    s.d2 = gs.d2 + I.r0;
    s.e = gs.e + I.r0;
    s.wy = gs.wy + I.r0;
    s.wu = gs.wu + I.r0;
    s.ly = gs.ly + I.r0;
    s.lu = gs.lu + I.r0;
    s.part = B.part.as<double>() + 3 * I.pb;
    s.partw = B.partw.as<int32_t>() + 4 * I.pb;
    s.partn = B.partn.as<int64_t>() + 2 * I.pb;
    s.out = B.out.as<double>() + 3 * m;
    s.outw = B.outw.as<int32_t>() + 4 * m;
    s.outn = B.outn.as<int64_t>() + 2 * m;
    s.flags = B.flags.as<int32_t>() + m;
    s.nb = I.nb;
    SP2Cfg &c = vc[m];
    c = SP2Cfg{};
    c.n_occ = P.n_occ;
    c.target2 = P.idem_target * P.idem_target;
    c.switch2 = P.switch_eta * P.switch_eta;
    c.max_iter = P.max_iter;
    c.tail = P.fp64_tail_steps;
    c.stall = P.stall_stop ? 1 : 0;
    c.mixed = I.mixed ? 1 : 0;
    c.span = 1;
    vh[m] = SP2Hist{B.h_trx.as<double>() + I.hoff,  B.h_trx2.as<double>() + I.hoff,
                    B.h_eta2.as<double>() + I.hoff, B.h_up.as<int8_t>() + I.hoff,
                    B.h_prec.as<int8_t>() + I.hoff, B.h_maxw.as<int32_t>() + I.hoff,
                    B.h_nnzx.as<int64_t>() + I.hoff, B.h_nnzy.as<int64_t>() + I.hoff};
    t64[m] = P.tau;
    t32[m] = (float)P.tau_fp32;
    SP2State &h = B.hs[m];
    std::memset(&h, 0, sizeof(h));
    h.status = ST_RUNNING;
    h.phase32 = I.mixed ? 1 : 0;
    h.cap = INT_MAX;
    h.sw = sw;
    h.nnz_cur = (int64_t)I.nnz0;
    h.once = P.prune_once ? 1 : 0;
    if (I.solo) {  // never enters the loop
      h.stop = 1;
      h.status = ST_FALLBACK;
    }
  }
  HIP_TRY(B.grp_inst.alloc(sizeof(int32_t) * B.ngroups));
  HIP_TRY(B.blk_inst.alloc(sizeof(int32_t) * B.nblocks));
  HIP_TRY(B.blk_local.alloc(sizeof(int32_t) * B.nblocks));
  HIP_TRY(B.inst_rows.alloc(sizeof(int32_t) * B.n));
  HIP_TRY(B.inst_r0.alloc(sizeof(int32_t) * B.n));
  HIP_TRY(B.ss.alloc(sizeof(StepScratch) * B.n));
  HIP_TRY(B.states.alloc(sizeof(SP2State) * B.n));
  HIP_TRY(B.cfgs.alloc(sizeof(SP2Cfg) * B.n));
  HIP_TRY(B.hists.alloc(sizeof(SP2Hist) * B.n));
  HIP_TRY(B.taus64.alloc(sizeof(double) * B.n));
  HIP_TRY(B.taus32.alloc(sizeof(float) * B.n));
  HIP_TRY(hipMemcpyAsync(B.grp_inst.p, gi.data(), sizeof(int32_t) * B.ngroups, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B.blk_inst.p, bi.data(), sizeof(int32_t) * B.nblocks, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B.blk_local.p, bl.data(), sizeof(int32_t) * B.nblocks, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B.inst_rows.p, ir.data(), sizeof(int32_t) * B.n, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B.inst_r0.p, i0.data(), sizeof(int32_t) * B.n, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B.ss.p, vs.data(), sizeof(StepScratch) * B.n, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B.cfgs.p, vc.data(), sizeof(SP2Cfg) * B.n, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B.hists.p, vh.data(), sizeof(SP2Hist) * B.n, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B.taus64.p, t64.data(), sizeof(double) * B.n, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B.taus32.p, t32.data(), sizeof(float) * B.n, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B.states.p, B.hs, sizeof(SP2State) * B.n, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));

  // ---- the loop: graphs of K iterations, K picked by timing the first replays ----
  int64_t max_iter_all = 0;
  for (const BatchInst &I : B.in) max_iter_all = std::max<int64_t>(max_iter_all, p[I.q].max_iter);
  const int poll_hint = p[B.in[0].q].poll_every;
  const int candidates[] = {2, 4, 8, 16};
  int K = poll_hint > 0 ? poll_hint : 0;  // 0: autotune (K, then the step kernel), unless cached
  int tune = 0;
  double best = 0.0;
  int bestK = 4;
  // after K: replays with the VALU kernel, the matrix cores, the VALU kernel
  // (the middle one against the mean of the two around it, which cancels the
  // steady growth of the rows), then the choice
  const int kernel_trials[] = {1, 0, 1};
  double trial_ms[3] = {0, 0, 0};
  bool trial_fair[3] = {false, false, false};
  int ktrial = 0;
  const std::string tkey = batch_tune_key(B.NT, B.SW, B.any32);
  bool kernel_tuned = K > 0;
  if (const char *force = std::getenv("ELLSP2_BATCH_KERNEL")) {  // a fixed step kernel (tests)
    if (force[0] == '0' || force[0] == '1') {
      B.kernel = force[0] - '0';
      kernel_tuned = true;
    }
  }
  if (K == 0 && !kernel_tuned) {
    BatchTune t;
    if (batch_tune_get(tkey, &t)) {
      K = t.K;
      B.kernel = t.kernel;
      kernel_tuned = true;
    }
  }
  hipEvent_t ta = nullptr, tb = nullptr;
  struct Ev2 {
    hipEvent_t &a, &b;
    ~Ev2()
    {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev2{ta, tb};
  HIP_TRY(hipEventCreate(&ta));
  HIP_TRY(hipEventCreate(&tb));
  const int64_t max_batches = max_iter_all + 128;
  for (int64_t batch = 0;; ++batch) {
    if (batch > max_batches) {
      g_last_error = "sp2_solve_batched: device control blocks did not reach a stop";
      return ELL_EDEVICE;
    }
    bool running = false;
    for (int m = 0; m < B.n; ++m) running = running || !B.hs[m].stop;
    if (!running) break;
    const bool tuning = K == 0 && tune < 4;
    const bool ktuning = !tuning && !kernel_tuned && ktrial < 3;
    if (ktuning) B.kernel = kernel_trials[ktrial];
    const int iters = K > 0 ? K : (tuning ? candidates[tune] : bestK);
    if (!B.exec || B.graph_iters != iters || B.graph_kernel != B.kernel) {
      int rc = B.capture(iters);
      if (rc) return rc;
    }
    std::vector<int> before(B.n);
    for (int m = 0; m < B.n; ++m) before[m] = B.hs[m].iter;
    HIP_TRY(hipEventRecord(ta, st));
    HIP_TRY(hipGraphLaunch(B.exec, st));
    HIP_TRY(hipEventRecord(tb, st));
    HIP_TRY(hipMemcpyAsync(B.hs, B.states.p, sizeof(SP2State) * B.n, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (tuning) {
      int adv = 0;
      for (int m = 0; m < B.n; ++m) adv = std::max(adv, B.hs[m].iter - before[m]);
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ta, tb));
      if (adv == iters) {  // every iteration of the graph did work: a fair sample
        const double per = ms / iters;
        if (tune == 0 || per < best) {
          best = per;
          bestK = iters;
        }
      }
      ++tune;
    } else if (ktuning) {
      int adv = 0;
      for (int m = 0; m < B.n; ++m) adv = std::max(adv, B.hs[m].iter - before[m]);
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ta, tb));
      trial_ms[ktrial] = ms / iters;
      trial_fair[ktrial] = adv == iters;
      if (++ktrial == 3) {
        // keep the matrix cores unless both VALU samples around them were fair and faster
        const bool valu = trial_fair[0] && trial_fair[1] && trial_fair[2] &&
                          0.5 * (trial_ms[0] + trial_ms[2]) < trial_ms[1];
        B.kernel = valu ? 1 : 0;
        kernel_tuned = true;
        batch_tune_put(tkey, BatchTune{bestK, B.kernel});
      }
    }
    // events of stopped instances
    bool dirty = false;
    int32_t need = 0;
    for (int m = 0; m < B.n; ++m) {
      SP2State &h = B.hs[m];
      if (!h.stop || h.status != ELL_EOVERFLOW) continue;
      need = std::max(need, h.need_width);
    }
    if (need > 0) {
      const int32_t nsw = roundup64(need);
      if (nsw > kMaxCap) {
        for (int m = 0; m < B.n; ++m)
          if (B.hs[m].stop && B.hs[m].status == ELL_EOVERFLOW) {
            B.in[m].solo = true;
            B.hs[m].status = ST_FALLBACK;
          }
      } else {
        int rc = batch_regrow(B, nsw);
        if (rc) return rc;
        for (int m = 0; m < B.n; ++m)
          if (B.hs[m].stop && B.hs[m].status == ELL_EOVERFLOW) {
            B.hs[m].stop = 0;
            B.hs[m].status = ST_RUNNING;
          }
      }
      dirty = true;
    }
    for (int m = 0; m < B.n; ++m) {
      SP2State &h = B.hs[m];
      if (!h.stop) continue;
      if (h.status == ST_SWITCH) {
        const BatchInst &I = B.in[m];
        HIP_TRY((launch_span_copy<float, double>(I.N, B.rows(B.A32, h.cur, I), B.rows(B.A64, 0, I), st)));
        h.cur = 0;
        h.phase32 = 0;
        h.stop = 0;
        h.status = ST_RUNNING;
        dirty = true;
      } else if (h.status == ST_FALLBACK) {
        B.in[m].solo = true;
      }
    }
    if (dirty) {
      HIP_TRY(hipMemcpyAsync(B.states.p, B.hs, sizeof(SP2State) * B.n, hipMemcpyHostToDevice, st));
      HIP_TRY(hipStreamSynchronize(st));
    }
  }
  HIP_TRY(hipEventRecord(t1, st));
  HIP_TRY(hipStreamSynchronize(st));
  float batch_ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&batch_ms, t0, t1));

  // ---- results ----
  std::vector<double> va(HT), vb(HT), vcc(HT);
  std::vector<int8_t> vu(HT), vp(HT);
  std::vector<int32_t> vw(HT);
  std::vector<int64_t> vx(HT), vy(HT);
  HIP_TRY(hipMemcpyAsync(va.data(), B.h_trx.p, sizeof(double) * HT, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(vb.data(), B.h_trx2.p, sizeof(double) * HT, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(vcc.data(), B.h_eta2.p, sizeof(double) * HT, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(vu.data(), B.h_up.p, HT, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(vp.data(), B.h_prec.p, HT, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(vw.data(), B.h_maxw.p, sizeof(int32_t) * HT, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(vx.data(), B.h_nnzx.p, sizeof(int64_t) * HT, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(vy.data(), B.h_nnzy.p, sizeof(int64_t) * HT, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  DevMem dw;
  HIP_TRY(dw.alloc(sizeof(int32_t)));
  for (int m = 0; m < B.n; ++m) {
    const BatchInst &I = B.in[m];
    if (I.solo) continue;
    const SP2State &h = B.hs[m];
    int32_t width = 0;
    int rc = h.phase32 ? batch_deliver<float>(B, B.A32, m, D[I.q], dw, &width)
                       : batch_deliver<double>(B, B.A64, m, D[I.q], dw, &width);
    const int status = rc ? rc : h.status;
    note(status);
    if (!r) continue;
    sp2_report_t &R = r[I.q];
    R.status = status;
    R.iterations = h.iter;
    R.final_M = rc == ELL_EOVERFLOW ? width : B.SW;
    R.eta = std::sqrt(h.eta2);
    R.trace_x = h.trx;
    R.seconds = batch_ms * 1e-3;
    R.batch_k = K > 0 ? K : bestK;
    R.batch_kernel = B.kernel;
    int f32 = 0;
    int64_t bytes = 0;
    for (int q = 0; q < h.iter; ++q) {
      const size_t o = (size_t)I.hoff + q;
      f32 += vp[o] ? 1 : 0;
      if (R.hist_trx) R.hist_trx[q] = va[o];
      if (R.hist_trx2) R.hist_trx2[q] = vb[o];
      if (R.hist_eta2) R.hist_eta2[q] = vcc[o];
      if (R.hist_up) R.hist_up[q] = vu[o];
      if (R.hist_prec) R.hist_prec[q] = vp[o];
      if (R.hist_maxw) R.hist_maxw[q] = vw[o];
      const int64_t sv = vp[o] ? 4 : 8;
      bytes += vx[o] * (sv + 4) + 4LL * I.N + vy[o] * (sv + 4) + 4LL * I.N;
    }
    R.fp32_iterations = f32;
    R.x2_bytes = bytes;
  }
  // instances the batch could not hold, each on its own
  for (int m = 0; m < B.n; ++m) {
    const BatchInst &I = B.in[m];
    if (!I.solo) continue;
    const int rc = sp2_solve(H[I.q], D[I.q], &p[I.q], r ? &r[I.q] : nullptr);
    note(rc);
  }
  return worst;
}

extern "C" const char *ellpack_strerror(int status)
{
  switch (status) {
    case ELL_OK: return "ok";
    case ELL_EINVAL: return "invalid argument";
    case ELL_ENOMEM: return "out of memory";
    case ELL_EOVERFLOW: return "row width exceeds capacity";
    case ELL_ENOCONV: return "no convergence";
    case ELL_EDEVICE: return "device error";
    case ELL_ENODEV: return "no device";
    case ELL_ENONFINITE: return "non-finite input";
    case ELL_EDEGENERATE: return "degenerate input";
    default: return "unknown status";
  }
}

extern "C" const char *ellpack_last_device_error(void) { return g_last_error.c_str(); }
