// Register-tiled X^2 for matrices whose rows are short column intervals
// (banded Hamiltonians and the density matrices SP2 makes from them).
//
// Inside the SP2 loop a matrix is held in span form: row i is stored densely
// over the columns [base[i], base[i] + len[i]) at val[i*SW ...], with zeros at
// the pruned positions inside the interval.  Stored ELLPACK entries are never
// exactly zero (they are kept only if |v| > tau >= 0), so the span form and the
// ELLPACK form describe the same matrix and convert into each other exactly.
//
// One wavefront computes G = 8 consecutive output rows.  Lane l of chunk r owns
// output column wlo + 64 r + l of all 8 rows, in registers acc[g][r].  For
// every chunk r the wave walks k in ascending order over the rows k whose
// interval meets the chunk, loads B = X[k][column] for its 64 columns with one
// coalesced load, and applies acc[g][r] = fma(X[i_g][k], B, acc[g][r]) for the
// 8 rows, the row value X[i_g][k] being the same for every lane (scalar
// loads).  Absent entries enter as zeros and a zero product leaves the
// accumulator unchanged, so every output entry is exactly the ascending-k
// chain of fused multiply-adds over the entries that exist: the same bits as
// the row-by-row sparse product.  A B load feeds 8 FMAs and no accumulator
// touches memory until the row is complete.
#include <algorithm>
#include <climits>
#include <cmath>

#include "band_common.h"
#include "ell_internal.h"
#include "../../include/ellsp2.h"

namespace ellsp2 {
namespace {

using namespace band;

constexpr int kG = kGroupRows;  // output rows per wave
constexpr int kWavesPerBlock = 4;
constexpr int kCP = 4;          // 64-column chunks accumulated per pass
constexpr int kKQ = 4;          // rows k held in registers per group: 64 kKQ
constexpr int kNormBlocks = 128;  // aligned 64-column blocks per row in the norm table
constexpr int kMaxChunks = 64;    // widest output window: 64 chunks of 64 columns

__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double absv(double a) { return __builtin_fabs(a); }
__device__ __forceinline__ float absv(float a) { return __builtin_fabsf(a); }

// X's values are never written while the kernel runs (X^2 and 2X - X^2 go to
// the other two buffers), so the row values X[i_g][k] -- the same for every
// lane -- are read through the scalar cache into SGPRs.
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ T sload(const T *p, ptrdiff_t off)
{
  return ((const_ptr<T>)p)[off];
}
__device__ __forceinline__ int sload_i(const int32_t *p, int off) { return ((const_ptr<int32_t>)p)[off]; }

// Raw buffer loads of row k of X: the buffer's range is exactly row k's
// interval, so lanes whose column lies outside it (either side: a negative
// byte offset wraps to a huge unsigned one) read 0 without any masking code.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const T *row, int len)
{
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(row), (short)0, len * (int)sizeof(T), kRawBufferFlags);
}
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, int off, double)
{
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int off, float)
{
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Rows of the group as seen by the accumulation: row g of the wave is X row
// i0 + g with interval [bs[g], bs[g] + ln[g]); `full` when all kG rows exist
// and are non-empty, and [ilo, ihi] is then the k range inside every interval.
struct GroupRows {
  int bs[kG], ln[kG];
  int i0, nrows, ilo, ihi;
  bool full;
};

// B of one row k for the CP chunks of a pass (zero outside row k's interval)
template <typename T, int CP>
__device__ __forceinline__ void load_row(const T *__restrict__ xv, const int SW, const int k, const int bk,
                                         const int lk, const int colb, T (&b)[CP])
{
  const __amdgpu_buffer_rsrc_t r = row_rsrc(xv + (size_t)k * SW, lk);
  const int off = colb - bk * (int)sizeof(T);
#pragma unroll
  for (int c = 0; c < CP; ++c) {
    // The whole byte offset goes in the VGPR: with the chunk's part folded into
    // the instruction's immediate offset, the 4-byte loads of this kernel gave
    // wrong values for some lanes on gfx950 (the range check and the address
    // did not agree).  The empty asm keeps the compiler from folding it back.
    int offc = off + c * kWave * (int)sizeof(T);
    asm volatile("" : "+v"(offc));
    b[c] = bload(r, offc, T(0));
  }
}

// acc[g][c] = sum over k in [klo, khi], ascending, of fma(X[i_g][k], X[k][col_c], .)
// for the CP chunks of the pass starting at column p0 (col_c = p0 + 64 c + lane).
// The B values of row k + 1 are loaded before row k is used.  k where some row
// of the group has no entry (the edges of the band, partial groups) take the
// masked path; inside every interval the row values are plain scalar loads
// from per-row pointers.  Positions outside an interval enter as exact zeros.
template <typename T, int CP>
__device__ __forceinline__ void accumulate(const T *__restrict__ xv, const int SW, const int32_t *xbase,
                                           const int32_t *xlen, const GroupRows &R, const int klo, const int khi,
                                           const int p0, T (&acc)[kG][kCP])
{
  const int lane = lane_id();
#pragma unroll
  for (int g = 0; g < kG; ++g)
#pragma unroll
    for (int c = 0; c < kCP; ++c) acc[g][c] = T(0);
  if (khi < klo) return;
  const int colb = (p0 + lane) * (int)sizeof(T);
  // interior k range of this pass
  const int jlo = R.full ? max(klo, R.ilo) : INT_MAX;
  const int jhi = R.full ? min(khi, R.ihi) : INT_MIN;
  T bn[CP];
  load_row<T, CP>(xv, SW, klo, sload_i(xbase, klo), sload_i(xlen, klo), colb, bn);
  int k = klo;
  // masked rows: left edge (and everything when there is no interior)
  auto masked = [&](int kend) {
    for (; k <= kend; ++k) {
      T bc[CP];
#pragma unroll
      for (int c = 0; c < CP; ++c) bc[c] = bn[c];
      if (k + 1 <= khi) load_row<T, CP>(xv, SW, k + 1, sload_i(xbase, k + 1), sload_i(xlen, k + 1), colb, bn);
#pragma unroll
      for (int g = 0; g < kG; ++g) {
        const int o = k - R.bs[g];
        const bool ok = g < R.nrows && (unsigned)o < (unsigned)R.ln[g];
        const T v = sload(xv, ok ? (ptrdiff_t)(R.i0 + g) * SW + o : (ptrdiff_t)R.i0 * SW);
        const T a = ok ? v : T(0);
#pragma unroll
        for (int c = 0; c < CP; ++c) acc[g][c] = fmadd(a, bc[c], acc[g][c]);
      }
    }
  };
  if (jlo <= jhi) {
    masked(jlo - 1);
    const T *rp[kG];
#pragma unroll
    for (int g = 0; g < kG; ++g) rp[g] = xv + (ptrdiff_t)(R.i0 + g) * SW - R.bs[g];
    for (; k <= jhi; ++k) {
      T bc[CP];
#pragma unroll
      for (int c = 0; c < CP; ++c) bc[c] = bn[c];
      if (k + 1 <= khi) load_row<T, CP>(xv, SW, k + 1, sload_i(xbase, k + 1), sload_i(xlen, k + 1), colb, bn);
#pragma unroll
      for (int g = 0; g < kG; ++g) {
        const T a = sload(rp[g], k);
#pragma unroll
        for (int c = 0; c < CP; ++c) acc[g][c] = fmadd(a, bc[c], acc[g][c]);
      }
    }
  }
  masked(khi);
}

// Per-row running state of the sweep, one lane per row (lane g holds row g).
__device__ __forceinline__ int row_get(int v, int g) { return __builtin_amdgcn_readlane(v, g); }
__device__ __forceinline__ int row_set(int v, int g, int x) { return lane_id() == g ? x : v; }

// One wave: output rows i0 .. i0 + nrows - 1, streamed 64 columns at a time.
// For every aligned 64-column chunk of the output window: accumulate the chunk
// of all 8 rows in registers (k ascending), then sweep it for each row --
// threshold, compaction of X^2 and 2X - X^2 (ELLPACK and/or span form), and
// the lane tree of the norm's squared differences for that aligned block.
// `once`: 2X - X^2 and the norm take the unpruned X^2 (one pruning per
// iteration); otherwise the pruned X^2.
template <typename T, bool WITH_U, bool OUT_ELL, bool OUT_SPAN>
__device__ void band_rows(const int N, const int i0, const int nrows, const SpanView<T> X, const SpanView<T> SY,
                          const SpanView<T> SU, const EllView<T> Y, const EllView<T> U, const T tau, const bool once,
                          const StepScratch &s, double *bsum, int32_t *fallback)
{
  const int lane = lane_id();
  const T *__restrict__ xv = X.val;
  const int SW = X.SW;

  // the 8 rows' intervals (uniform)
  int bs[kG], ln[kG];
#pragma unroll
  for (int g = 0; g < kG; ++g) {
    const bool ok = g < nrows;
    bs[g] = ok ? uni(X.base[i0 + g]) : 0;
    ln[g] = ok ? uni(X.len[i0 + g]) : 0;
  }
  int kmin = INT_MAX, kmax = -1;
#pragma unroll
  for (int g = 0; g < kG; ++g)
    if (ln[g] > 0) {
      kmin = min(kmin, bs[g]);
      kmax = max(kmax, bs[g] + ln[g] - 1);
    }
  if (kmax < 0) {
    // every row of the group is empty: so are its rows of X^2 and 2X - X^2.
    // (Handled first: no index arithmetic may start from kmin = INT_MAX.)
    if (lane == 0) {
      for (int g = 0; g < nrows; ++g) {
        const int i = i0 + g;
        if (OUT_ELL) Y.nnz[i] = 0;
        if (OUT_ELL && WITH_U) U.nnz[i] = 0;
        if (OUT_SPAN) {
          SY.base[i] = 0;
          SY.len[i] = 0;
          if (WITH_U) {
            SU.base[i] = 0;
            SU.len[i] = 0;
          }
        }
        s.wy[i] = 0;
        s.wu[i] = 0;
        if (s.ly) s.ly[i] = 0;
        if (s.lu) s.lu[i] = 0;
        s.d1[i] = 0.0;
        s.d2[i] = 0.0;
        s.e[i] = 0.0;
      }
    }
    return;
  }
  // intervals of the rows k in [kmin, kmax], lane-distributed: k = kmin + 64 q + lane
  int kbq[kKQ], klq[kKQ];
#pragma unroll
  for (int q = 0; q < kKQ; ++q) {
    const int k = kmin + q * kWave + lane;
    const bool ok = k <= kmax;
    klq[q] = ok ? X.len[k] : 0;
    kbq[q] = ok ? X.base[k] : 0;
  }
  const bool kfit = kmax - kmin < kKQ * kWave;  // every row k is in registers
  // output window: every row k's interval and the rows' own intervals,
  // widened to whole aligned 64-column blocks
  int wlo = kmin, whi = kmax;
  if (kfit) {
#pragma unroll
    for (int q = 0; q < kKQ; ++q)
      if (klq[q] > 0) {
        wlo = min(wlo, kbq[q]);
        whi = max(whi, kbq[q] + klq[q] - 1);
      }
  } else {
    for (int k0 = kmin; k0 <= kmax; k0 += kWave) {
      const int k = k0 + lane;
      if (k <= kmax) {
        const int l = X.len[k];
        if (l > 0) {
          const int b = X.base[k];
          wlo = min(wlo, b);
          whi = max(whi, b + l - 1);
        }
      }
    }
  }
  wlo = wmin(wlo) & ~63;
  whi = wmax(whi);
  const int nchunk = (whi - wlo + kWave) / kWave;
  if (nchunk > kMaxChunks) {
    if (lane == 0) atomicOr(fallback, 1);
    return;
  }
  const int b0 = (wlo >> 6) & ~63;  // first block of the norm's 128-block table

  // running state, lane g = row g
  int st_cy = 0, st_cu = 0, st_yf = INT_MAX, st_yl = -1, st_uf = INT_MAX, st_ul = -1;
  for (int r = lane; r < kG * kNormBlocks; r += kWave) bsum[r] = 0.0;

  GroupRows R;
  R.i0 = i0;
  R.nrows = nrows;
  R.full = nrows == kG;
  R.ilo = INT_MIN;
  R.ihi = INT_MAX;
#pragma unroll
  for (int g = 0; g < kG; ++g) {
    R.bs[g] = bs[g];
    R.ln[g] = ln[g];
    R.full = R.full && ln[g] > 0;
    R.ilo = max(R.ilo, bs[g]);
    R.ihi = min(R.ihi, bs[g] + ln[g] - 1);
  }

  for (int pc = 0; pc < nchunk; pc += kCP) {
    const int cnt = min(kCP, nchunk - pc);
    const int p0 = wlo + pc * kWave;         // first column of the pass
    const int p1 = p0 + cnt * kWave - 1;     // last column of the pass
    // rows k whose interval meets the pass: a conservative k range
    int klo = INT_MAX, khi = -1;
    if (kfit) {
#pragma unroll
      for (int q = 0; q < kKQ; ++q) {
        const bool meet = klq[q] > 0 && kbq[q] <= p1 && kbq[q] + klq[q] - 1 >= p0;
        const uint64_t m = __ballot(meet);
        if (m) {
          klo = min(klo, kmin + q * kWave + (int)__builtin_ctzll(m));
          khi = max(khi, kmin + q * kWave + 63 - (int)__builtin_clzll(m));
        }
      }
    } else {
      for (int k0 = kmin; k0 <= kmax; k0 += kWave) {
        const int k = k0 + lane;
        bool meet = false;
        if (k <= kmax) {
          const int l = X.len[k];
          const int b = X.base[k];
          meet = l > 0 && b <= p1 && b + l - 1 >= p0;
        }
        const uint64_t m = __ballot(meet);
        if (m) {
          klo = min(klo, k0 + (int)__builtin_ctzll(m));
          khi = max(khi, k0 + 63 - (int)__builtin_clzll(m));
        }
      }
    }
    klo = uni(klo);
    khi = uni(khi);
    T acc[kG][kCP];
    switch (cnt) {
      case 1: accumulate<T, 1>(xv, SW, X.base, X.len, R, klo, khi, p0, acc); break;
      case 2: accumulate<T, 2>(xv, SW, X.base, X.len, R, klo, khi, p0, acc); break;
      case 3: accumulate<T, 3>(xv, SW, X.base, X.len, R, klo, khi, p0, acc); break;
      default: accumulate<T, 4>(xv, SW, X.base, X.len, R, klo, khi, p0, acc); break;
    }
#pragma unroll
    for (int cc = 0; cc < kCP; ++cc) {
    if (cc >= cnt) break;
    const int c0 = p0 + cc * kWave;  // first column of the chunk
    const int col = c0 + lane;
    // sweep the chunk for every row
    const int rel = (c0 >> 6) - b0;
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      if (g >= nrows) break;
      const int i = i0 + g;
      const T y = acc[g][cc];
      const int ox = col - bs[g];
      const T x = (unsigned)ox < (unsigned)ln[g] ? xv[(size_t)i * SW + ox] : T(0);
      if (col == i) {  // X_ii and the unpruned (X.X)_ii
        s.d1[i] = (double)x;
        s.d2[i] = (double)y;
      }
      const bool ky = absv(y) > tau;
      const T yk = ky ? y : T(0);
      const T ym = once ? y : yk;  // the X^2 value 2X - X^2 and the norm see
      const uint64_t my = __ballot(ky);
      int cy = row_get(st_cy, g);
      if (OUT_ELL && ky) {
        const int pos = cy + lanes_below(my);
        if (pos < Y.M) {
          Y.idx[(size_t)i * Y.M + pos] = col;
          Y.val[(size_t)i * Y.M + pos] = y;
        }
      }
      st_cy = row_set(st_cy, g, cy + __popcll(my));
      int yf = row_get(st_yf, g);
      if (my) {
        yf = min(yf, c0 + (int)__builtin_ctzll(my));
        st_yf = row_set(st_yf, g, yf);
        st_yl = row_set(st_yl, g, c0 + 63 - (int)__builtin_clzll(my));
      }
      if (OUT_SPAN && yf != INT_MAX) {
        const int o = col - yf;
        if ((unsigned)o < (unsigned)SY.SW) SY.val[(size_t)i * SY.SW + o] = yk;
      }
      if (WITH_U) {
        const T v = T(2) * x - ym;
        const bool ku = absv(v) > tau;
        const uint64_t mu = __ballot(ku);
        const int cu = row_get(st_cu, g);
        if (OUT_ELL && ku) {
          const int pos = cu + lanes_below(mu);
          if (pos < U.M) {
            U.idx[(size_t)i * U.M + pos] = col;
            U.val[(size_t)i * U.M + pos] = v;
          }
        }
        st_cu = row_set(st_cu, g, cu + __popcll(mu));
        int uf = row_get(st_uf, g);
        if (mu) {
          uf = min(uf, c0 + (int)__builtin_ctzll(mu));
          st_uf = row_set(st_uf, g, uf);
          st_ul = row_set(st_ul, g, c0 + 63 - (int)__builtin_clzll(mu));
        }
        if (OUT_SPAN && uf != INT_MAX) {
          const int o = col - uf;
          if ((unsigned)o < (unsigned)SU.SW) SU.val[(size_t)i * SU.SW + o] = ku ? v : T(0);
        }
      }
      const double dd = (double)ym - (double)x;
      const double t = wave_tree(dd * dd);
      if (lane == 0 && rel < kNormBlocks) bsum[g * kNormBlocks + rel] = t;
    }
    }
  }

  // finish every row
  wave_sync();
#pragma unroll 1
  for (int g = 0; g < nrows; ++g) {
    const int i = i0 + g;
    // norm row term: blocks b0 .. b0 + 127 form two perfect 64-block subtrees
    const double g0 = wave_tree(bsum[g * kNormBlocks + lane]);
    const double g1 = wave_tree(bsum[g * kNormBlocks + kWave + lane]);
    const int cy = row_get(st_cy, g), cu = row_get(st_cu, g);
    const int yf = row_get(st_yf, g), yl = row_get(st_yl, g);
    const int uf = row_get(st_uf, g), ul = row_get(st_ul, g);
    const int ylen = yl >= 0 ? yl - yf + 1 : 0;
    const int ulen = ul >= 0 ? ul - uf + 1 : 0;
    if (lane == 0) {
      if (OUT_ELL) Y.nnz[i] = min(cy, Y.M);
      if (OUT_ELL && WITH_U) U.nnz[i] = min(cu, U.M);
      if (OUT_SPAN) {
        SY.base[i] = ylen ? yf : 0;
        SY.len[i] = ylen;
        if (WITH_U) {
          SU.base[i] = ulen ? uf : 0;
          SU.len[i] = ulen;
        }
      }
      s.wy[i] = cy;
      s.wu[i] = WITH_U ? cu : 0;
      if (s.ly) s.ly[i] = ylen;
      if (s.lu) s.lu[i] = WITH_U ? ulen : 0;
      s.e[i] = g0 + g1;
      if (i < wlo || i >= wlo + nchunk * kWave) {  // column i never swept
        s.d1[i] = 0.0;
        s.d2[i] = 0.0;
      }
    }
  }
}

template <typename T, bool WITH_U, bool OUT_ELL, bool OUT_SPAN>
__global__ __launch_bounds__(256) void k_x2_band(int N, SpanRot3<T> spans, Rot3<T> ells, const SP2State *st,
                                                 T tau, StepScratch s, int32_t *fallback)
{
  __shared__ double bsum_s[kWavesPerBlock][kG * kNormBlocks];
  int cur = 0;
  bool once = false;
  if (st) {
    if (st->stop) return;
    cur = st->cur;
    once = st->once != 0;
  }
  const int w = uni(threadIdx.x >> 6);
  const int grp = xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + w;
  const int i0 = grp * kG;
  if (i0 >= N) return;
  const int nrows = min(kG, N - i0);
  const int cy = cur == 2 ? 0 : cur + 1, cu = cur == 0 ? 2 : cur - 1;
  band_rows<T, WITH_U, OUT_ELL, OUT_SPAN>(N, i0, nrows, spans.b[cur], spans.b[cy], spans.b[cu], ells.b[cy],
                                          ells.b[cu], tau, once, s, bsum_s[w], fallback);
}

// Batched form: the instances' rows are stacked in one span matrix, instance m
// from row r0[m] (a multiple of kG), with its own local column numbers.  Row
// group grp belongs to instance grp_inst[grp]; the wave works on that instance's
// rows as a matrix of its own (views shifted by r0), so every row, its column
// blocks and the norm's tree see exactly the coordinates of a single solve.
// The instance's state selects the buffers, whether it still runs, and its
// precision; the launch for one precision skips instances in the other.
template <typename T>
__device__ __forceinline__ SpanView<T> shift_rows(SpanView<T> v, int r0)
{
  v.val += (size_t)r0 * v.SW;
  v.base += r0;
  v.len += r0;
  return v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_x2_band_batch(int ngroups, SpanRot3<T> spans, const int32_t *grp_inst,
                                                       const int32_t *inst_r0, const int32_t *inst_rows,
                                                       const SP2State *states, int32_t phase32, const T *taus,
                                                       const StepScratch *ss, int32_t *flags)
{
  __shared__ double bsum_s[kWavesPerBlock][kG * kNormBlocks];
  const int w = uni(threadIdx.x >> 6);
  const int grp = xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + w;
  if (grp >= ngroups) return;
  const int m = uni(grp_inst[grp]);
  const SP2State *st = states + m;
  if (st->stop || st->phase32 != phase32) return;
  const int cur = uni(st->cur);
  const int cy = cur == 2 ? 0 : cur + 1, cu = cur == 0 ? 2 : cur - 1;
  const int r0 = uni(inst_r0[m]), n = uni(inst_rows[m]);
  const int i0 = grp * kG - r0;
  if (i0 >= n) return;  // alignment rows after the instance's last row
  const EllView<T> none{nullptr, nullptr, nullptr, 0};
  band_rows<T, true, false, true>(n, i0, min(kG, n - i0), shift_rows(spans.b[cur], r0), shift_rows(spans.b[cy], r0),
                                  shift_rows(spans.b[cu], r0), none, none, taus[m], st->once != 0, ss[m], bsum_s[w],
                                  flags + m);
}

// ---- conversions between ELLPACK and span form -----------------------------------------

// Interval length of every row of an ELLPACK matrix, and a flag if any stored
// value is exactly zero (the span form cannot represent it; with flags null
// the values are not read).
template <typename T>
__global__ __launch_bounds__(256) void k_ell_extent(int N, EllView<T> A, int32_t *len, int32_t *flags,
                                                    int32_t *maxlen, unsigned long long *sums)
{
  __shared__ int32_t wl[kWavesPerBlock];
  __shared__ unsigned long long ws[2][kWavesPerBlock];
  const int i = blockIdx.x * 256 + threadIdx.x;
  int l = 0, n = 0;
  if (i < N) {
    n = A.nnz[i];
    if (n > 0) l = A.idx[(size_t)i * A.M + n - 1] - A.idx[(size_t)i * A.M] + 1;
    if (len) len[i] = l;
    if (flags) {  // (null: the caller knows the matrix stores no zero)
      bool zero = false;
      for (int q = 0; q < n; ++q) zero |= A.val[(size_t)i * A.M + q] == T(0);
      if (zero) atomicOr(flags, 4);
    }
  }
  if (!maxlen) return;  // the same for the whole launch
  unsigned long long sn = (unsigned long long)n, sl = (unsigned long long)l;
  for (int o = 32; o > 0; o >>= 1) {
    sn += __shfl_xor(sn, o, kWave);
    sl += __shfl_xor(sl, o, kWave);
  }
  l = wmax(l);
  if (lane_id() == 0) {
    wl[threadIdx.x >> 6] = l;
    ws[0][threadIdx.x >> 6] = sn;
    ws[1][threadIdx.x >> 6] = sl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMax(maxlen, max(max(wl[0], wl[1]), max(wl[2], wl[3])));
    if (sums) {
      atomicAdd(&sums[0], ws[0][0] + ws[0][1] + ws[0][2] + ws[0][3]);
      atomicAdd(&sums[1], ws[1][0] + ws[1][1] + ws[1][2] + ws[1][3]);
    }
  }
}

// ELLPACK -> span form, one wave per row: positions not stored are zero.
// The interval starts on a multiple of `align` columns (a power of two) and
// holds a multiple of `align` positions.
template <typename T>
__global__ __launch_bounds__(256) void k_ell_to_span(int N, EllView<T> A, SpanView<T> S, int align)
{
  const int w = threadIdx.x >> 6;
  const int i = blockIdx.x * kWavesPerBlock + w;
  if (i >= N) return;
  const int lane = lane_id();
  const int n = A.nnz[i];
  const int32_t *ci = A.idx + (size_t)i * A.M;
  const T *vi = A.val + (size_t)i * A.M;
  const int b = n > 0 ? ci[0] & ~(align - 1) : 0;
  const int l = n > 0 ? ((ci[n - 1] | (align - 1)) + 1) - b : 0;
  // each lane writes its stored entries and the zeros up to the next one
  // (columns are sorted and unique); lane 0 also the zeros before the first
  T *row = S.val + (size_t)i * S.SW;
  for (int q = lane; q < n; q += kWave) {
    const int c = ci[q] - b;
    row[c] = vi[q];
    const int next = q + 1 < n ? ci[q + 1] - b : l;
    for (int p = c + 1; p < next; ++p) row[p] = T(0);
  }
  if (lane == 0)
    for (int p = 0; p < (n > 0 ? ci[0] - b : 0); ++p) row[p] = T(0);
  if (lane == 0) {
    S.base[i] = b;
    S.len[i] = l;
  }
}

// span form -> ELLPACK (nonzero positions, ascending), one wave per row, the
// waves striding over the rows; up to four 64-position chunks of a row are
// loaded before they are compacted.  The widest row goes to *wmax with one
// atomic per workgroup, skipped when the stored maximum is already as wide.
template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_span_to_ell(int N, SpanView<TS> S, EllView<TD> A, int32_t *wmax)
{
  __shared__ int32_t bmax;
  if (threadIdx.x == 0) bmax = 0;
  __syncthreads();
  const int lane = lane_id();
  int cmax = 0;
  for (int i = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); i < N; i += gridDim.x * kWavesPerBlock) {
    const int b = S.base[i], l = S.len[i];
    int c = 0;
    for (int p1 = 0; p1 < l; p1 += 4 * kWave) {
      TS v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p = p1 + u * kWave + lane;
        v[u] = p < l ? S.val[(size_t)i * S.SW + p] : TS(0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p0 = p1 + u * kWave;
        if (p0 >= l) break;  // (the same for the whole wave)
        const bool keep = v[u] != TS(0);
        const uint64_t m = __ballot(keep);
        if (keep) {
          const int pos = c + lanes_below(m);
          if (pos < A.M) {
            A.idx[(size_t)i * A.M + pos] = b + p0 + lane;
            A.val[(size_t)i * A.M + pos] = (TD)v[u];
          }
        }
        c += __popcll(m);
      }
    }
    if (lane == 0) A.nnz[i] = min(c, A.M);
    cmax = max(cmax, c);
  }
  if (wmax) {
    if (lane == 0) atomicMax(&bmax, cmax);
    __syncthreads();
    if (threadIdx.x == 0 && bmax > __hip_atomic_load(wmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(wmax, bmax);
  }
}

// span copy between strides and precisions (float -> double is exact)
template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_span_copy(int N, SpanView<TS> S, SpanView<TD> D)
{
  const int w = threadIdx.x >> 6;
  const int i = blockIdx.x * kWavesPerBlock + w;
  if (i >= N) return;
  const int l = S.len[i];
  for (int p = lane_id(); p < l; p += kWave) D.val[(size_t)i * D.SW + p] = (TD)S.val[(size_t)i * S.SW + p];
  if (lane_id() == 0) {
    D.base[i] = S.base[i];
    D.len[i] = l;
  }
}

}  // namespace

// ---- launchers ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_x2_band(int N, SpanRot3<T> spans, Rot3<T> ells, const SP2State *st, bool with_u, bool out_ell,
                          T tau, const StepScratch &s, int32_t *fallback, hipStream_t stream)
{
  const int groups = (N + kG - 1) / kG;
  const dim3 grid((groups + kWavesPerBlock - 1) / kWavesPerBlock), block(256);
  if (out_ell) {
    if (with_u)
      hipLaunchKernelGGL((k_x2_band<T, true, true, false>), grid, block, 0, stream, N, spans, ells, st, tau, s,
                         fallback);
    else
      hipLaunchKernelGGL((k_x2_band<T, false, true, false>), grid, block, 0, stream, N, spans, ells, st, tau, s,
                         fallback);
  } else {
    if (x2_band16_fits(N, spans.b[0].SW, (int)sizeof(T)))
      return launch_x2_band16<T>(N, spans, st, tau, s, fallback, stream);
    hipLaunchKernelGGL((k_x2_band<T, true, false, true>), grid, block, 0, stream, N, spans, ells, st, tau, s,
                       fallback);
  }
  return hipGetLastError();
}
template hipError_t launch_x2_band<double>(int, SpanRot3<double>, Rot3<double>, const SP2State *, bool, bool,
                                           double, const StepScratch &, int32_t *, hipStream_t);
template hipError_t launch_x2_band<float>(int, SpanRot3<float>, Rot3<float>, const SP2State *, bool, bool, float,
                                          const StepScratch &, int32_t *, hipStream_t);

template <typename T>
hipError_t launch_x2_band_batch(int ngroups, SpanRot3<T> spans, const int32_t *grp_inst, const int32_t *inst_r0,
                                const int32_t *inst_rows, const SP2State *states, int32_t phase32, const T *taus,
                                const StepScratch *ss, int32_t *flags, hipStream_t stream, bool matrix_cores,
                                bool sym)
{
  static_assert(kBatchAlign % kGroupRows == 0, "batch alignment is a whole number of row groups");
  if (matrix_cores && x2_band16_fits(ngroups * kGroupRows, spans.b[0].SW, (int)sizeof(T)))
    return launch_x2_band16_batch<T>(ngroups * kGroupRows / 16, spans, grp_inst, inst_r0, inst_rows, states, phase32,
                                     taus, ss, flags, sym, stream);
  const dim3 grid((ngroups + kWavesPerBlock - 1) / kWavesPerBlock), block(256);
  hipLaunchKernelGGL((k_x2_band_batch<T>), grid, block, 0, stream, ngroups, spans, grp_inst, inst_r0, inst_rows,
                     states, phase32, taus, ss, flags);
  return hipGetLastError();
}
template hipError_t launch_x2_band_batch<double>(int, SpanRot3<double>, const int32_t *, const int32_t *,
                                                 const int32_t *, const SP2State *, int32_t, const double *,
                                                 const StepScratch *, int32_t *, hipStream_t, bool, bool);
template hipError_t launch_x2_band_batch<float>(int, SpanRot3<float>, const int32_t *, const int32_t *,
                                                const int32_t *, const SP2State *, int32_t, const float *,
                                                const StepScratch *, int32_t *, hipStream_t, bool, bool);

template <typename T>
hipError_t launch_ell_extent(int N, EllView<T> A, int32_t *len, int32_t *flags, int32_t *maxlen,
                             unsigned long long *sums, hipStream_t stream)
{
  hipLaunchKernelGGL((k_ell_extent<T>), dim3((N + 255) / 256), dim3(256), 0, stream, N, A, len, flags, maxlen, sums);
  return hipGetLastError();
}
template hipError_t launch_ell_extent<double>(int, EllView<double>, int32_t *, int32_t *, int32_t *,
                                              unsigned long long *, hipStream_t);
template hipError_t launch_ell_extent<float>(int, EllView<float>, int32_t *, int32_t *, int32_t *,
                                             unsigned long long *, hipStream_t);

template <typename T>
hipError_t launch_ell_to_span(int N, EllView<T> A, SpanView<T> S, hipStream_t stream, int align)
{
  if (align < 1 || (align & (align - 1))) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_ell_to_span<T>), dim3((N + kWavesPerBlock - 1) / kWavesPerBlock), dim3(256), 0, stream, N,
                     A, S, align);
  return hipGetLastError();
}
template hipError_t launch_ell_to_span<double>(int, EllView<double>, SpanView<double>, hipStream_t, int);
template hipError_t launch_ell_to_span<float>(int, EllView<float>, SpanView<float>, hipStream_t, int);

template <typename TS, typename TD>
hipError_t launch_span_to_ell(int N, SpanView<TS> S, EllView<TD> A, int32_t *wmax, hipStream_t stream)
{
  const int blocks = std::min((N + kWavesPerBlock - 1) / kWavesPerBlock, 1024);
  hipLaunchKernelGGL((k_span_to_ell<TS, TD>), dim3(std::max(blocks, 1)), dim3(256), 0, stream, N, S, A, wmax);
  return hipGetLastError();
}
template hipError_t launch_span_to_ell<double, double>(int, SpanView<double>, EllView<double>, int32_t *,
                                                       hipStream_t);
template hipError_t launch_span_to_ell<float, double>(int, SpanView<float>, EllView<double>, int32_t *,
                                                      hipStream_t);
template hipError_t launch_span_to_ell<float, float>(int, SpanView<float>, EllView<float>, int32_t *, hipStream_t);

template <typename TS, typename TD>
hipError_t launch_span_copy(int N, SpanView<TS> S, SpanView<TD> D, hipStream_t stream)
{
  hipLaunchKernelGGL((k_span_copy<TS, TD>), dim3((N + kWavesPerBlock - 1) / kWavesPerBlock), dim3(256), 0, stream, N,
                     S, D);
  return hipGetLastError();
}
template hipError_t launch_span_copy<double, double>(int, SpanView<double>, SpanView<double>, hipStream_t);
template hipError_t launch_span_copy<float, float>(int, SpanView<float>, SpanView<float>, hipStream_t);
template hipError_t launch_span_copy<float, double>(int, SpanView<float>, SpanView<double>, hipStream_t);

}  // namespace ellsp2
