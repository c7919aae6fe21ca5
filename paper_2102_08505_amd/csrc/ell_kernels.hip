// Device kernels of libellsp2 for gfx950 (CDNA4, wave64).
//
// The hot kernel is k_x2_step: one wavefront per output row i.  The wave
// computes the column window [lo, hi] that row i of X.X can touch (the union
// of the column ranges of every row k referenced by row i, plus row i's own
// columns), zeroes an LDS accumulator over it, and runs Gustavson's row
// product: k in ascending order over row i, the 64 lanes over the entries of
// row k, one fused multiply-add per entry into the LDS accumulator.  Every
// accumulator entry therefore receives its products in ascending k with one
// rounding each, which is the bit-exact reading of the X^2 step (the entries
// of one row k have distinct columns, so lanes never collide, and LDS
// operations of one wave complete in program order).  The window is then
// swept in ascending column order, 64 columns per step, and a ballot plus a
// masked bit count compacts the surviving entries (|v| > tau) into the output
// row; the same sweep forms 2X - X^2 over the union of the two patterns and
// the squared differences of the idempotency norm, whose per-row pairwise
// tree is built 64 entries at a time with a butterfly over the lanes.
//
// Row spans wider than the window are processed in several passes over
// consecutive column windows; every pass re-reads the rows k and keeps only
// the entries of its window, so the result does not depend on the window.
#include <climits>
#include <cmath>

#include "ell_internal.h"
#include "../../include/ellsp2.h"

namespace ellsp2 {
namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kWin = 512;        // accumulator window per wave (entries)
constexpr int kRing = 128;       // two 64-entry blocks of squared differences
constexpr int kMaxBlocks = 128;  // 64-entry blocks of one row's union list

__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int lanes_below(uint64_t m)
{
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ void wave_sync()
{
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int wave_min(int v)
{
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ int wave_max(int v)
{
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
  return v;
}

// Perfect binary tree over the 64 lanes, lane pairs (0,1), (2,3), ... first.
// The sum is valid in lane 0.
__device__ __forceinline__ double wave_tree(double v)
{
  for (int s = 1; s < kWave; s <<= 1) v = v + __shfl_down(v, s, kWave);
  return v;
}

__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double absv(double a) { return __builtin_fabs(a); }
__device__ __forceinline__ float absv(float a) { return __builtin_fabsf(a); }

// Perfect tree over 1024 values held 4 per thread by a 256-thread block;
// valid in every thread on return.
__device__ double block_tree_1024(double a0, double a1, double a2, double a3, double *ws)
{
  double v = (a0 + a1) + (a2 + a3);
  v = wave_tree(v);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) ws[w] = v;
  __syncthreads();
  double r = (ws[0] + ws[1]) + (ws[2] + ws[3]);
  __syncthreads();
  return r;
}

// --------------------------------------------------------------------------
// the fused X^2 / trace / norm / update row kernel
// --------------------------------------------------------------------------
template <typename T, bool WITH_U>
__device__ void x2_row(const int i, const int32_t *__restrict__ xnnz, const int32_t *__restrict__ xidx,
                       const T *__restrict__ xval, const int M, EllView<T> Y, EllView<T> U, const T tau,
                       T *acc, T *xw, uint8_t *xp, double *ring, double *bsum, const StepScratch &s)
{
  const int lane = lane_id();
  const int wi = uniform_i(xnnz[i]);
  const int32_t *ci = xidx + (size_t)i * M;
  const T *vi = xval + (size_t)i * M;

  // window bounds and the diagonal entry X_ii
  int lo = INT_MAX, hi = -1;
  double d1 = 0.0;
  bool has_diag = false;
  for (int s0 = 0; s0 < wi; s0 += kWave) {
    const int sl = s0 + lane;
    if (sl < wi) {
      const int k = ci[sl];
      const int nk = xnnz[k];
      int f = k, l = k;
      if (nk > 0) {
        const int32_t *ck = xidx + (size_t)k * M;
        f = min(f, ck[0]);
        l = max(l, ck[nk - 1]);
      }
      lo = min(lo, f);
      hi = max(hi, l);
      if (k == i) {
        has_diag = true;
        d1 = (double)vi[sl];
      }
    }
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  const uint64_t dm = __ballot(has_diag);
  if (dm) d1 = __shfl(d1, __builtin_ctzll(dm), kWave);

  int cy = 0, cu = 0, nu = 0;
  double d2 = 0.0;
  for (int wlo = lo; wlo <= hi; wlo += kWin) {
    const int wlen = min(kWin, hi - wlo + 1);
    for (int p = lane; p < wlen; p += kWave) {
      acc[p] = T(0);
      xp[p] = 0;
    }
    for (int s0 = 0; s0 < wi; s0 += kWave) {
      const int sl = s0 + lane;
      if (sl < wi) {
        const int p = ci[sl] - wlo;
        if ((unsigned)p < (unsigned)wlen) {
          xw[p] = vi[sl];
          xp[p] = 1;
        }
      }
    }
    wave_sync();
    // Gustavson: k ascending over row i, the lanes over row k
    for (int sk = 0; sk < wi; ++sk) {
      const int k = uniform_i(ci[sk]);
      const T a = vi[sk];
      const int nk = uniform_i(xnnz[k]);
      const int32_t *ck = xidx + (size_t)k * M;
      const T *vk = xval + (size_t)k * M;
      for (int t = lane; t < nk; t += kWave) {
        const int p = ck[t] - wlo;
        if ((unsigned)p < (unsigned)wlen) acc[p] = fmadd(a, vk[t], acc[p]);
      }
    }
    wave_sync();
    if (i >= wlo && i < wlo + wlen) d2 = (double)acc[i - wlo];
    // ascending sweep: compaction of X^2 and 2X - X^2, squared differences
    for (int q0 = 0; q0 < wlen; q0 += kWave) {
      const int p = q0 + lane;
      const bool in = p < wlen;
      const int j = wlo + p;
      const T y = in ? acc[p] : T(0);
      const bool ky = in && absv(y) > tau;
      const bool hx = in && xp[p] != 0;
      const T x = hx ? xw[p] : T(0);
      const uint64_t my = __ballot(ky);
      if (ky) {
        const int pos = cy + lanes_below(my);
        if (pos < Y.M) {
          Y.idx[(size_t)i * Y.M + pos] = j;
          Y.val[(size_t)i * Y.M + pos] = y;
        }
      }
      cy += __popcll(my);
      const T yk = ky ? y : T(0);
      if (WITH_U) {
        const T v = T(2) * x - yk;
        const bool ku = in && absv(v) > tau;
        const uint64_t mu = __ballot(ku);
        if (ku) {
          const int pos = cu + lanes_below(mu);
          if (pos < U.M) {
            U.idx[(size_t)i * U.M + pos] = j;
            U.val[(size_t)i * U.M + pos] = v;
          }
        }
        cu += __popcll(mu);
      }
      const bool un = ky || hx;
      const uint64_t mn = __ballot(un);
      if (un) {
        const double dd = (double)yk - (double)x;
        ring[(nu + lanes_below(mn)) & (kRing - 1)] = dd * dd;
      }
      const int nu_next = nu + __popcll(mn);
      if ((nu_next >> 6) != (nu >> 6)) {
        wave_sync();
        const int b = nu >> 6;
        const double t = wave_tree(ring[((b & 1) << 6) + lane]);
        if (lane == 0 && b < kMaxBlocks) bsum[b] = t;
      }
      nu = nu_next;
    }
  }
  // the last, partial block of the union list, then the tree over block sums
  wave_sync();
  if (nu & 63) {
    const int b = nu >> 6;
    const double v = lane < (nu & 63) ? ring[((b & 1) << 6) + lane] : -0.0;
    const double t = wave_tree(v);
    if (lane == 0 && b < kMaxBlocks) bsum[b] = t;
  }
  wave_sync();
  const int nb = (nu + 63) >> 6;
  double ev = 0.0;
  if (nb > kMaxBlocks) {
    ev = __builtin_nan("");  // row wider than the supported union length
  } else if (nb > 0) {
    const double v0 = wave_tree(lane < nb ? bsum[lane] : -0.0);
    const double v1 = wave_tree(lane + kWave < nb ? bsum[lane + kWave] : -0.0);
    ev = nb > kWave ? v0 + v1 : v0;
  }
  if (lane == 0) {
    Y.nnz[i] = min(cy, Y.M);
    s.wy[i] = cy;
    if (WITH_U) {
      U.nnz[i] = min(cu, U.M);
      s.wu[i] = cu;
    } else {
      s.wu[i] = 0;
    }
    s.d1[i] = d1;
    s.d2[i] = d2;
    s.e[i] = ev;
  }
}

template <typename T, bool WITH_U>
__global__ __launch_bounds__(256) void k_x2_step(int N, Rot3<T> bufs, const SP2State *st, T tau,
                                                 StepScratch s)
{
  __shared__ T acc_s[kWavesPerBlock][kWin];
  __shared__ T xw_s[kWavesPerBlock][kWin];
  __shared__ uint8_t xp_s[kWavesPerBlock][kWin];
  __shared__ double ring_s[kWavesPerBlock][kRing];
  __shared__ double bsum_s[kWavesPerBlock][kMaxBlocks];
  int cur = 0;
  if (st) {
    if (st->stop) return;
    cur = st->cur;
  }
  const int w = uniform_i(threadIdx.x >> 6);
  const int i = blockIdx.x * kWavesPerBlock + w;
  if (i >= N) return;
  const EllView<T> X = bufs.b[cur];
  const EllView<T> Y = bufs.b[cur == 2 ? 0 : cur + 1];
  const EllView<T> U = bufs.b[cur == 0 ? 2 : cur - 1];
  x2_row<T, WITH_U>(i, X.nnz, X.idx, X.val, X.M, Y, U, tau, acc_s[w], xw_s[w], xp_s[w], ring_s[w],
                    bsum_s[w], s);
}

// --------------------------------------------------------------------------
// deterministic reductions of the step outputs
// --------------------------------------------------------------------------
struct Nnz3 {
  const int32_t *p[3];
};

__global__ __launch_bounds__(256) void k_step_partial(int N, const SP2State *st, StepScratch s, Nnz3 nz)
{
  __shared__ double ws[4];
  __shared__ int32_t wsi[2][4];
  __shared__ long long wsl[2][4];
  if (st && st->stop) return;
  const int cur = st ? st->cur : 0;
  const int32_t *nx = nz.p[cur];
  const int32_t *ny = nz.p[cur == 2 ? 0 : cur + 1];
  const int base = blockIdx.x * kRedBlock + threadIdx.x * 4;
  double a[3][4];
  int32_t wy = 0, wu = 0;
  long long sx = 0, sy = 0;
  for (int q = 0; q < 4; ++q) {
    const int r = base + q;
    const bool in = r < N;
    a[0][q] = in ? s.d1[r] : -0.0;
    a[1][q] = in ? s.d2[r] : -0.0;
    a[2][q] = in ? s.e[r] : -0.0;
    if (in) {
      wy = max(wy, s.wy[r]);
      wu = max(wu, s.wu[r]);
      if (nx) sx += nx[r];
      if (ny) sy += ny[r];
    }
  }
  double t[3];
  for (int c = 0; c < 3; ++c) t[c] = block_tree_1024(a[c][0], a[c][1], a[c][2], a[c][3], ws);
  for (int o = 32; o > 0; o >>= 1) {
    wy = max(wy, __shfl_xor(wy, o, kWave));
    wu = max(wu, __shfl_xor(wu, o, kWave));
    sx += __shfl_xor(sx, o, kWave);
    sy += __shfl_xor(sy, o, kWave);
  }
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    wsi[0][w] = wy;
    wsi[1][w] = wu;
    wsl[0][w] = sx;
    wsl[1][w] = sy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = 0; c < 3; ++c) s.part[c * s.nb + blockIdx.x] = t[c];
    s.partw[blockIdx.x] = max(max(wsi[0][0], wsi[0][1]), max(wsi[0][2], wsi[0][3]));
    s.partw[s.nb + blockIdx.x] = max(max(wsi[1][0], wsi[1][1]), max(wsi[1][2], wsi[1][3]));
    s.partn[blockIdx.x] = wsl[0][0] + wsl[0][1] + wsl[0][2] + wsl[0][3];
    s.partn[s.nb + blockIdx.x] = wsl[1][0] + wsl[1][1] + wsl[1][2] + wsl[1][3];
  }
}

// Final level: perfect tree over the nb partials (padded with -0.0, the exact
// additive identity), so the result equals the pairwise tree over all rows.
__device__ void final_reduce(const StepScratch &s, double *ws)
{
  const int base = threadIdx.x * 4;
  for (int c = 0; c < 3; ++c) {
    double a[4];
    for (int q = 0; q < 4; ++q) a[q] = base + q < s.nb ? s.part[c * s.nb + base + q] : -0.0;
    const double t = block_tree_1024(a[0], a[1], a[2], a[3], ws);
    if (threadIdx.x == 0) s.out[c] = t;
  }
  if (threadIdx.x == 0) {
    int32_t wy = 0, wu = 0;
    long long sx = 0, sy = 0;
    for (int b = 0; b < s.nb; ++b) {
      wy = max(wy, s.partw[b]);
      wu = max(wu, s.partw[s.nb + b]);
      sx += s.partn[b];
      sy += s.partn[s.nb + b];
    }
    s.outw[0] = wy;
    s.outw[1] = wu;
    s.outn[0] = sx;
    s.outn[1] = sy;
  }
}

__device__ bool stalled(const double *h, int n)
{
  if (n < 3) return false;
  if (!(h[n - 3] < 1e-4)) return false;
  const double now = h[n] < h[n - 1] ? h[n] : h[n - 1];
  const double before = h[n - 2] < h[n - 3] ? h[n - 2] : h[n - 3];
  return now >= before;
}

// One decision of the SP2 loop, taken on the device by a single thread.
__device__ void decide(SP2State *st, const SP2Cfg &cfg, const SP2Hist &h, const StepScratch &s)
{
  const int n = st->iter;
  const double trx = s.out[0], trx2 = s.out[1], eta2 = s.out[2];
  st->trx = trx;
  st->trx2 = trx2;
  st->eta2 = eta2;
  st->wy_max = s.outw[0];
  st->wu_max = s.outw[1];
  h.trx[n] = trx;
  h.trx2[n] = trx2;
  h.eta2[n] = eta2;
  h.maxw[n] = s.outw[0];
  h.prec[n] = (int8_t)st->phase32;
  h.up[n] = -1;
  h.nnzx[n] = s.outn[0];
  h.nnzy[n] = s.outn[1];
  const bool stall = cfg.stall && stalled(h.eta2 + st->phase_start, n - st->phase_start);
  if (st->phase32) {
    if (eta2 < cfg.switch2 || stall) {
      st->phase_start = n + 1;
      st->iter = n + 1;
      st->stop = 1;
      st->status = (n + 1 == cfg.max_iter) ? ELL_ENOCONV : ST_SWITCH;
      return;
    }
  } else {
    if (eta2 < cfg.target2 && st->fp64_updates >= (cfg.mixed ? cfg.tail : 0)) {
      st->status = ELL_OK;
      st->stop = 1;
      st->iter = n + 1;
      return;
    }
    if (stall) {
      st->status = ELL_ENOCONV;
      st->stop = 1;
      st->iter = n + 1;
      return;
    }
  }
  if (n + 1 == cfg.max_iter) {
    st->status = ELL_ENOCONV;
    st->stop = 1;
    st->iter = n + 1;
    return;
  }
  const double a = fabs(2.0 * trx - trx2 - cfg.n_occ);
  const double b = fabs(trx2 - cfg.n_occ);
  const bool up = a < b;
  const int need = up ? s.outw[1] : s.outw[0];
  if (need > st->cap) {
    st->status = ELL_EOVERFLOW;
    st->need_width = need;
    st->stop = 1;
    return;
  }
  h.up[n] = up ? 1 : 0;
  const int c = st->cur;
  st->cur = up ? (c == 0 ? 2 : c - 1) : (c == 2 ? 0 : c + 1);
  if (!st->phase32) st->fp64_updates += 1;
  st->iter = n + 1;
}

__global__ __launch_bounds__(256) void k_step_final(SP2State *st, SP2Cfg cfg, SP2Hist h, StepScratch s)
{
  __shared__ double ws[4];
  if (st && st->stop) return;
  final_reduce(s, ws);
  __syncthreads();
  if (st && threadIdx.x == 0) decide(st, cfg, h, s);
}

// --------------------------------------------------------------------------
// initialisation: Gershgorin bounds and X0
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gersh_rows(int N, EllView<double> H, double *plo, double *phi,
                                                    int32_t *flags)
{
  __shared__ double slo[256], shi[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double lo = INFINITY, hi = -INFINITY;
  if (i < N) {
    double r = 0.0, hii = 0.0;
    bool bad = false;
    const int n = H.nnz[i];
    for (int q = 0; q < n; ++q) {
      const int j = H.idx[(size_t)i * H.M + q];
      const double h = H.val[(size_t)i * H.M + q];
      if (!isfinite(h)) bad = true;
      if (j == i) hii = h;
      else r = r + fabs(h);
    }
    if (bad) atomicOr(flags, 2);
    lo = hii - r;
    hi = hii + r;
  }
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + o]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    plo[blockIdx.x] = slo[0];
    phi[blockIdx.x] = shi[0];
  }
}

__global__ __launch_bounds__(256) void k_gersh_final(int nb, const double *plo, const double *phi, double *out)
{
  __shared__ double slo[256], shi[256];
  double lo = INFINITY, hi = -INFINITY;
  for (int b = threadIdx.x; b < nb; b += 256) {
    lo = fmin(lo, plo[b]);
    hi = fmax(hi, phi[b]);
  }
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + o]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = slo[0];
    out[1] = shi[0];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_x0(int N, EllView<double> H, EllView<T> X, double emax, double inv,
                                            T tau, int32_t *wmax)
{
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int n = H.nnz[i];
  const int32_t *ci = H.idx + (size_t)i * H.M;
  const double *vi = H.val + (size_t)i * H.M;
  int c = 0, q = 0;
  bool diag_done = false;
  while (q < n || !diag_done) {
    int j;
    double h;
    if (q < n && (diag_done || ci[q] <= i)) {
      j = ci[q];
      h = vi[q];
      ++q;
    } else {
      j = i;
      h = 0.0;
    }
    if (j == i) diag_done = true;
    const double x = (j == i) ? (emax - h) * inv : (-h) * inv;
    const T xt = (T)x;
    if (absv(xt) > tau) {
      if (c < X.M) {
        X.idx[(size_t)i * X.M + c] = j;
        X.val[(size_t)i * X.M + c] = xt;
      }
      ++c;
    }
  }
  X.nnz[i] = min(c, X.M);
  atomicMax(wmax, c);
}

// Row copy between capacities and precisions (widening float -> double is exact).
template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_copy(int N, EllView<TS> src, EllView<TD> dst)
{
  const int w = threadIdx.x >> 6;
  const int i = blockIdx.x * kWavesPerBlock + w;
  if (i >= N) return;
  const int n = min(src.nnz[i], dst.M);
  for (int q = lane_id(); q < n; q += kWave) {
    dst.idx[(size_t)i * dst.M + q] = src.idx[(size_t)i * src.M + q];
    dst.val[(size_t)i * dst.M + q] = (TD)src.val[(size_t)i * src.M + q];
  }
  if (lane_id() == 0) dst.nnz[i] = n;
}

template <typename T>
__global__ __launch_bounds__(256) void k_validate(int N, EllView<T> A, int32_t *flags)
{
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int n = A.nnz[i];
  if (n < 0 || n > A.M) {
    atomicOr(flags, 1);
    return;
  }
  int prev = -1;
  bool bad = false, nonfinite = false;
  for (int q = 0; q < n; ++q) {
    const int j = A.idx[(size_t)i * A.M + q];
    if (j < 0 || j >= N || j <= prev) bad = true;
    prev = j;
    if (!isfinite((double)A.val[(size_t)i * A.M + q])) nonfinite = true;
  }
  if (bad) atomicOr(flags, 1);
  if (nonfinite) atomicOr(flags, 2);
}

template <typename T>
__global__ __launch_bounds__(256) void k_trace_rows(int N, EllView<T> A, double *d)
{
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  double v = 0.0;
  const int n = A.nnz[i];
  for (int q = 0; q < n; ++q)
    if (A.idx[(size_t)i * A.M + q] == i) v = (double)A.val[(size_t)i * A.M + q];
  d[i] = v;
}

__global__ __launch_bounds__(256) void k_tree_partial(int n, const double *d, double *part)
{
  __shared__ double ws[4];
  const int base = blockIdx.x * kRedBlock + threadIdx.x * 4;
  double a[4];
  for (int q = 0; q < 4; ++q) a[q] = base + q < n ? d[base + q] : -0.0;
  const double t = block_tree_1024(a[0], a[1], a[2], a[3], ws);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

}  // namespace

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
template <typename T>
hipError_t launch_x2_step(int N, Rot3<T> bufs, const SP2State *st, bool with_u, T tau,
                          const StepScratch &s, hipStream_t stream)
{
  const dim3 grid((N + kWavesPerBlock - 1) / kWavesPerBlock), block(256);
  if (with_u)
    hipLaunchKernelGGL((k_x2_step<T, true>), grid, block, 0, stream, N, bufs, st, tau, s);
  else
    hipLaunchKernelGGL((k_x2_step<T, false>), grid, block, 0, stream, N, bufs, st, tau, s);
  return hipGetLastError();
}
template hipError_t launch_x2_step<double>(int, Rot3<double>, const SP2State *, bool, double,
                                           const StepScratch &, hipStream_t);
template hipError_t launch_x2_step<float>(int, Rot3<float>, const SP2State *, bool, float,
                                          const StepScratch &, hipStream_t);

hipError_t launch_reduce(int N, const SP2State *st, const StepScratch &s, hipStream_t stream,
                         const int32_t *nnz0, const int32_t *nnz1, const int32_t *nnz2)
{
  Nnz3 nz{{nnz0, nnz1, nnz2}};
  hipLaunchKernelGGL(k_step_partial, dim3(s.nb), dim3(256), 0, stream, N, st, s, nz);
  return hipGetLastError();
}

hipError_t launch_decide(SP2State *st, SP2Cfg cfg, SP2Hist hist, const StepScratch &s, hipStream_t stream)
{
  hipLaunchKernelGGL(k_step_final, dim3(1), dim3(256), 0, stream, st, cfg, hist, s);
  return hipGetLastError();
}

hipError_t launch_final_only(const StepScratch &s, hipStream_t stream)
{
  SP2Cfg cfg{};
  SP2Hist h{};
  hipLaunchKernelGGL(k_step_final, dim3(1), dim3(256), 0, stream, (SP2State *)nullptr, cfg, h, s);
  return hipGetLastError();
}

hipError_t launch_gershgorin(int N, EllView<double> H, double *rowlo, double *rowhi, double *emin_emax,
                             int32_t *flags, hipStream_t stream)
{
  const int nb = (N + 255) / 256;
  hipLaunchKernelGGL(k_gersh_rows, dim3(nb), dim3(256), 0, stream, N, H, rowlo, rowhi, flags);
  hipLaunchKernelGGL(k_gersh_final, dim3(1), dim3(256), 0, stream, nb, rowlo, rowhi, emin_emax);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_x0(int N, EllView<double> H, EllView<T> X, double emax, double inv, T tau, int32_t *wmax,
                     hipStream_t stream)
{
  hipLaunchKernelGGL((k_x0<T>), dim3((N + 255) / 256), dim3(256), 0, stream, N, H, X, emax, inv, tau, wmax);
  return hipGetLastError();
}
template hipError_t launch_x0<double>(int, EllView<double>, EllView<double>, double, double, double,
                                      int32_t *, hipStream_t);
template hipError_t launch_x0<float>(int, EllView<double>, EllView<float>, double, double, float, int32_t *,
                                     hipStream_t);

template <typename TS, typename TD>
hipError_t launch_copy(int N, EllView<TS> src, EllView<TD> dst, hipStream_t stream)
{
  hipLaunchKernelGGL((k_copy<TS, TD>), dim3((N + kWavesPerBlock - 1) / kWavesPerBlock), dim3(256), 0, stream,
                     N, src, dst);
  return hipGetLastError();
}
template hipError_t launch_copy<double, double>(int, EllView<double>, EllView<double>, hipStream_t);
template hipError_t launch_copy<float, float>(int, EllView<float>, EllView<float>, hipStream_t);
template hipError_t launch_copy<float, double>(int, EllView<float>, EllView<double>, hipStream_t);

template <typename T>
hipError_t launch_validate(int N, EllView<T> A, int32_t *flags, hipStream_t stream)
{
  hipLaunchKernelGGL((k_validate<T>), dim3((N + 255) / 256), dim3(256), 0, stream, N, A, flags);
  return hipGetLastError();
}
template hipError_t launch_validate<double>(int, EllView<double>, int32_t *, hipStream_t);
template hipError_t launch_validate<float>(int, EllView<float>, int32_t *, hipStream_t);

template <typename T>
hipError_t launch_trace_rows(int N, EllView<T> A, double *d, hipStream_t stream)
{
  hipLaunchKernelGGL((k_trace_rows<T>), dim3((N + 255) / 256), dim3(256), 0, stream, N, A, d);
  return hipGetLastError();
}
template hipError_t launch_trace_rows<double>(int, EllView<double>, double *, hipStream_t);
template hipError_t launch_trace_rows<float>(int, EllView<float>, double *, hipStream_t);

// Pairwise tree over n doubles: 1024-element blocks, then one more level over
// the block sums (n <= 1024 * 1024).  `part` holds ceil(n/1024) doubles.
hipError_t launch_tree_sum(int n, const double *d, double *part, double *out, hipStream_t stream)
{
  const int nb = (n + kRedBlock - 1) / kRedBlock;
  hipLaunchKernelGGL(k_tree_partial, dim3(nb), dim3(256), 0, stream, n, d, part);
  hipLaunchKernelGGL(k_tree_partial, dim3(1), dim3(256), 0, stream, nb, part, out);
  return hipGetLastError();
}

}  // namespace ellsp2
