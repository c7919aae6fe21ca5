// X^2 of span-form matrices on the matrix cores, FP64 and FP32: the product,
// pruning, and per-row outputs of every SP2 iteration (the "SP2 Loop X2",
// "SP2 Loop Norm" and "SP2 Loop Misc" steps of the paper's section
// "Performance Evaluation using an ExaSP2 Application", on the ELLPACK
// matrix-matrix multiply of its section "Performance Evaluation using System
// Matrices").
//
// In span form row i of X is stored densely over the columns
// [base[i], base[i] + len[i]) at val[i*SW ...], with zeros at the pruned
// positions inside the interval.  Around the diagonal, X^2 is then a product of
// narrow dense strips.  One wavefront computes 16 consecutive output rows.  Its
// window of output columns is cut into aligned 64-column blocks; each block is
// four 16x16 tiles, accumulated with v_mfma_f64_16x16x4_f64 (FP32:
// v_mfma_f32_16x16x4_f32) over the rows k whose interval meets the block, k
// ascending four at a time.
//
// Both matrix instructions form each element as a chain of fused multiply-adds
// in ascending k, rounded to the working precision at every step (k = 0..3
// inside one instruction, instructions issued in ascending k): the chain of the
// row-by-row sparse product.
// Positions outside an interval enter as exact zeros and a zero product leaves
// the accumulator unchanged, so every entry of X^2 has the bits of the sparse
// product's ascending-k chain over the entries that exist.
//
// The sweep of a block -- threshold, span output of X^2 and 2X - X^2, the
// norm's squared differences -- works in the tile layout: lane l holds column
// l % 16 of four rows (FP64: rows l / 16 + 4 t; FP32: rows 4 (l / 16) + t, for
// t = 0..3), so a row's 16 columns of one tile are one 16-lane row of the
// wavefront.
#include <climits>

#include "band_common.h"
#include "span16_common.h"
#include "ell_internal.h"
#include "sp2_decide.h"

namespace ellsp2 {
namespace {

using namespace band;
using namespace span16;

constexpr int kR = 16;                  // output rows per wave (the tile's rows)
constexpr int kP = 4;                   // 16-column tiles per 64-column block
constexpr int kWpb = 4;                 // waves per workgroup
constexpr int kKQ = 4;                  // rows k whose intervals are held in registers: 64 kKQ
constexpr int kMeta = kKQ * kWave;      // entries of the wave's LDS table of row intervals
constexpr int kLev = 16;                // levels of the norm's block tree (2^16 aligned 64-column blocks)

// This lane's row's kept columns of a block from the four tiles' wave masks.
__device__ __forceinline__ void row_bits(const uint64_t (&m)[4], int q, uint32_t &lo, uint32_t &hi)
{
  lo = seg16(m[0], q) | seg16(m[1], q) << 16;
  hi = seg16(m[2], q) | seg16(m[3], q) << 16;
}

// Span output of one tile of one row, lane column col: the columns from the
// row's first kept one up to the block's last kept one (lastw).
template <typename T>
__device__ __forceinline__ void put(__amdgpu_buffer_rsrc_t rs, int first, int lastw, int col, int row0, int SW,
                                    bool act, T v)
{
  const int o = col - first;
  st(rs, at<T>(act && col <= lastw && (unsigned)o < (unsigned)SW, row0 + o), v);
}
// Zeros for the columns gap_lo .. c0 - 1 of a row (blocks that kept nothing
// after its last kept column, followed by one that keeps something).
template <typename T>
__device__ void fill_gap(__amdgpu_buffer_rsrc_t rs, int first, int gap_lo, int c0, int r, int row0, int SW, bool act)
{
  for (int c = gap_lo + r; c < c0; c += 16) {
    const int o = c - first;
    st(rs, at<T>(act && (unsigned)o < (unsigned)SW, row0 + o), T(0));
  }
}

// Accumulate one 64-column block: acc[p] += X[i0 .. i0+15][k] X[k][p0 + 16 p ..]
// over k = klo .. khi, four k per step (a step past khi multiplies zeros);
// tile p takes part only in the steps that meet its own range tlo[p] .. thi[p].
// A operand: lane (r, q) = (l % 16, l / 16) supplies X[i0 + r][k0 + q] -- with
// SYMA (X bitwise symmetric) read as X[k0 + q][i0 + r] from row k's interval,
// four 128-byte runs per load instead of sixteen rows of 32 bytes;
// B operand: lane (r, q) supplies X[k0 + q][p0 + 16 p + r].
// Two operand sets alternate: the loads of step k0 + 4 are in flight while
// the products of step k0 issue.  Every load is range-checked (rows k past
// khi have no entry in the block's columns, and rows k past kmax have an
// empty interval in the table), so the step after the last needs no branch.
template <typename T, bool LDS_META, bool SYMA>
__device__ __forceinline__ void mma_block(const SpanView<T> &X, const __amdgpu_buffer_rsrc_t xr, const int2 *meta,
                                          const int kmin, const int kmax, const int klo, const int khi,
                                          const int (&tlo)[kP], const int (&thi)[kP], const int p0, const int arow,
                                          const int bA, const int lA, const int ai,
                                          typename Mfma<T>::acc (&acc)[kP])
{
  const int lane = lane_id();
  const int r = lane & 15, q = lane >> 4;
  const int SW = X.SW;
  auto interval = [&](int k0) {  // interval of row k0 + q
    const int k = k0 + q;
    int2 m;
    if (LDS_META) {
      m = meta[k - kmin];
    } else {
      const int kc = min(k, kmax);
      m.x = X.base[kc];
      m.y = k <= kmax ? X.len[kc] : 0;
    }
    return m;
  };
  auto load = [&](int k0, int2 m, T &a, T (&b)[kP]) {
    const int k = k0 + q;
    const int brow = k * SW - m.x;
    if (SYMA)
      a = ld(xr, at<T>((unsigned)(ai - m.x) < (unsigned)m.y, brow + ai), T(0));
    else
      a = ld(xr, at<T>((unsigned)(k - bA) < (unsigned)lA, arow + k), T(0));
#pragma unroll
    for (int p = 0; p < kP; ++p) {
      const int col = p0 + 16 * p + r;
      b[p] = ld(xr, at<T>((unsigned)(col - m.x) < (unsigned)m.y, brow + col), T(0));
    }
  };
  // In FP64, tile p's products are skipped at steps outside its own k range
  // (its B operand is all zeros there).  FP32 products are cheap enough that
  // the branches cost more than the products they skip: all four issue, adding
  // exact zeros.
  auto mma = [&](int k0, T a, const T (&b)[kP]) {
#pragma unroll
    for (int p = 0; p < kP; ++p)
      if (sizeof(T) == 4 || (k0 <= thi[p] && k0 + 3 >= tlo[p])) acc[p] = Mfma<T>::mma(a, b[p], acc[p]);
  };
  const int nsteps = (khi - klo) / 4 + 1;
  T a0, b0[kP], a1, b1[kP];
  load(klo, interval(klo), a0, b0);
  int2 m1 = interval(klo + 4);
  int k0 = klo;
  // (the scheduling barriers keep each set's loads ahead of the other set's products)
  for (int st2 = 0; st2 + 2 <= nsteps; st2 += 2, k0 += 8) {
    load(k0 + 4, m1, a1, b1);
    const int2 m0 = interval(k0 + 8);
    __builtin_amdgcn_sched_barrier(0);
    mma(k0, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    load(k0 + 8, m0, a0, b0);
    m1 = interval(k0 + 12);
    __builtin_amdgcn_sched_barrier(0);
    mma(k0 + 4, a1, b1);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (nsteps & 1) mma(k0, a0, b0);
}

// One wave: output rows i0 .. i0 + nrows - 1 (nrows <= 16) of X^2 and 2X - X^2.
// `once`: 2X - X^2 and the norm take the unpruned X^2 (one pruning per
// iteration); otherwise the pruned X^2.  SYMA: X is bitwise symmetric (the A
// operand is read through the symmetry).  WITH_U false: a standalone product
// without the 2X - X^2 output (SU is neither read nor written; its widths
// read 0).
template <typename T, bool SYMA = false, bool WITH_U = true>
__device__ void rows16(const int N, const int i0, const int nrows, const SpanView<T> X, const SpanView<T> SY,
                       const SpanView<T> SU, const T tau, const bool once, const StepScratch &s, double *stk,
                       double *sq, int2 *meta, [[maybe_unused]] int32_t *fallback)
{
  const int lane = lane_id();
  const int r = lane & 15, q = lane >> 4;
  // the three matrices share one row stride (they rotate roles every iteration)
  const int SW = X.SW;
  const int bytes = N * SW * (int)sizeof(T);  // < 2^31: the launcher takes this kernel only then
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(X.val, (short)0, bytes, kRawBufferFlags);
  const __amdgpu_buffer_rsrc_t yr = __builtin_amdgcn_make_buffer_rsrc(SY.val, (short)0, bytes, kRawBufferFlags);
  const __amdgpu_buffer_rsrc_t ur = __builtin_amdgcn_make_buffer_rsrc(SU.val, (short)0, bytes, kRawBufferFlags);

  // interval of row r (lane l holds row l % 16)
  const int bA = r < nrows ? X.base[i0 + r] : 0;
  const int lA = r < nrows ? X.len[i0 + r] : 0;
  const int kmin = wmin(lA > 0 ? bA : INT_MAX);
  const int kmax = wmax(lA > 0 ? bA + lA - 1 : -1);
  if (kmax < 0) {
    // every row of the group is empty, and so are its rows of X^2 and 2X - X^2
    if (q == 0 && r < nrows) {
      const int i = i0 + r;
      SY.base[i] = 0;
      SY.len[i] = 0;
      if (WITH_U) {
        SU.base[i] = 0;
        SU.len[i] = 0;
      }
      s.wy[i] = 0;
      s.wu[i] = 0;
      if (s.ly) s.ly[i] = 0;
      if (s.lu) s.lu[i] = 0;
      s.d1[i] = 0.0;
      s.d2[i] = 0.0;
      s.e[i] = 0.0;
    }
    return;
  }
  // intervals of the rows k in [kmin, kmax], lane-distributed: k = kmin + 64 j + lane
  int kbq[kKQ], klq[kKQ];
#pragma unroll
  for (int j = 0; j < kKQ; ++j) {
    const int k = kmin + j * kWave + lane;
    const bool ok = k <= kmax;
    klq[j] = ok ? X.len[k] : 0;
    kbq[j] = ok ? X.base[k] : 0;
  }
  // the table holds rows kmin .. kmin + kMeta - 1 (empty past kmax); the
  // accumulation reads up to 15 rows past the last row k it uses
  const bool kfit = kmax - kmin < kMeta - 16;
  // output window: the rows' own intervals and every row k's interval, from
  // an aligned 64-column block on
  int wlo = kmin, whi = kmax;
  if (kfit) {
#pragma unroll
    for (int j = 0; j < kKQ; ++j)
      if (klq[j] > 0) {
        wlo = min(wlo, kbq[j]);
        whi = max(whi, kbq[j] + klq[j] - 1);
      }
  } else {
    for (int k0 = kmin; k0 <= kmax; k0 += kWave) {
      const int k = k0 + lane;
      if (k <= kmax) {
        const int l = X.len[k];
        if (l > 0) {
          wlo = min(wlo, X.base[k]);
          whi = max(whi, X.base[k] + l - 1);
        }
      }
    }
  }
  wlo = wmin(wlo) & ~63;
  whi = wmax(whi);
  const int nblk = (whi - wlo + kWave) / kWave;
  const int b_first = wlo >> 6;  // the window's first aligned block
  if (kfit) {
#pragma unroll
    for (int j = 0; j < kKQ; ++j) meta[j * kWave + lane] = make_int2(kbq[j], klq[j]);
    wave_sync();
  }

  // this lane's output rows
  int bC[4], lC[4], xrow[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int rr = Mfma<T>::row(q, t);
    bC[t] = __shfl(bA, rr, kWave);
    lC[t] = __shfl(lA, rr, kWave);
    xrow[t] = (i0 + rr) * SW - bC[t];
  }
  const int arow = (i0 + r) * SW - bA;
  RowRun ry[4], ru[4];
  // the norm's pending subtrees of row lane / 4 (lanes 4 g): bit l set when
  // stk[g][l] holds a completed left subtree of 2^l blocks awaiting its right
  // sibling
  uint32_t pend = 0;

  for (int pc = 0; pc < nblk; ++pc) {
    const int p0 = wlo + pc * kWave;
    // rows k whose interval meets each tile of the block, and the block
    int tlo[kP], thi[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
      tlo[p] = INT_MAX;
      thi[p] = -1;
    }
    auto meet = [&](int kbase, int b, int l) {
#pragma unroll
      for (int p = 0; p < kP; ++p) {
        const int c0 = p0 + 16 * p;
        const uint64_t m = __ballot(l > 0 && b <= c0 + 15 && b + l - 1 >= c0);
        if (m) {
          tlo[p] = min(tlo[p], kbase + (int)__builtin_ctzll(m));
          thi[p] = max(thi[p], kbase + 63 - (int)__builtin_clzll(m));
        }
      }
    };
    if (kfit) {
#pragma unroll
      for (int j = 0; j < kKQ; ++j) meet(kmin + j * kWave, kbq[j], klq[j]);
    } else {
      for (int k0 = kmin; k0 <= kmax; k0 += kWave) {
        const int k = k0 + lane;
        const bool in = k <= kmax;
        meet(k0, in ? X.base[k] : 0, in ? X.len[k] : 0);
      }
    }
    int klo = INT_MAX, khi = -1;
#pragma unroll
    for (int p = 0; p < kP; ++p) {
      tlo[p] = uni(tlo[p]);
      thi[p] = uni(thi[p]);
      klo = min(klo, tlo[p]);
      khi = max(khi, thi[p]);
    }
    // X at the block's output positions, for 2X - X^2 and the norm: loaded
    // first, so the loads complete under the block's products
    T xv[4][kP];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int p = 0; p < kP; ++p) {
        const int col = p0 + 16 * p + r;
        xv[t][p] = ld(xr, at<T>((unsigned)(col - bC[t]) < (unsigned)lC[t], xrow[t] + col), T(0));
      }
    typename Mfma<T>::acc acc[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) acc[p] = typename Mfma<T>::acc{T(0), T(0), T(0), T(0)};
    if (klo <= khi) {
      if (kfit) mma_block<T, true, SYMA>(X, xr, meta, kmin, kmax, klo, khi, tlo, thi, p0, arow, bA, lA, i0 + r, acc);
      else mma_block<T, false, SYMA>(X, xr, meta, kmin, kmax, klo, khi, tlo, thi, p0, arow, bA, lA, i0 + r, acc);
    }

    // sweep the block, row quad by row quad
    const bool diag = p0 <= i0 + kR - 1 && p0 + kWave - 1 >= i0;  // a diagonal entry lies in the block
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int rr = Mfma<T>::row(q, t);
      const int i = i0 + rr;
      const bool act = rr < nrows;
      T yk[kP], uk[kP];
      bool ky[kP], ku[kP];
      double e[kP];
#pragma unroll
      for (int p = 0; p < kP; ++p) {
        const T y = acc[p][t], x = xv[t][p];
        ky[p] = act && absv(y) > tau;
        yk[p] = ky[p] ? y : T(0);
        const T ym = once ? y : yk[p];  // the X^2 value 2X - X^2 and the norm see
        const T v = T(2) * x - ym;
        ku[p] = WITH_U && act && absv(v) > tau;
        uk[p] = ku[p] ? v : T(0);
        const double d = (double)ym - (double)x;
        e[p] = d * d;
      }
      uint64_t my[kP], mu[kP];
#pragma unroll
      for (int p = 0; p < kP; ++p) {
        my[p] = __ballot(ky[p]);
        mu[p] = WITH_U ? __ballot(ku[p]) : 0;
      }
      // (a quad whose rows keep nothing of X^2, or of 2X - X^2, in this block
      // leaves that output's row state as it is and writes nothing to it)
      uint32_t lo, hi;
      int gy = p0, gu = p0;
      if ((my[0] | my[1] | my[2] | my[3]) != 0) {
        row_bits(my, q, lo, hi);
        const int ly = ry[t].add(lo, hi, p0, gy);
#pragma unroll
        for (int p = 0; p < kP; ++p) put<T>(yr, ry[t].first, ly, p0 + 16 * p + r, i * SW, SW, act, yk[p]);
      }
      if (WITH_U && (mu[0] | mu[1] | mu[2] | mu[3]) != 0) {
        row_bits(mu, q, lo, hi);
        const int lu = ru[t].add(lo, hi, p0, gu);
#pragma unroll
        for (int p = 0; p < kP; ++p) put<T>(ur, ru[t].first, lu, p0 + 16 * p + r, i * SW, SW, act, uk[p]);
      }
      // the norm's squared differences, to the block table [row][column]
#pragma unroll
      for (int p = 0; p < kP; ++p) sq[rr * kWave + 16 * p + r] = e[p];
      if (__ballot(gy < p0 || gu < p0)) {
        fill_gap<T>(yr, ry[t].first, gy, p0, r, i * SW, SW, act);
        if (WITH_U) fill_gap<T>(ur, ru[t].first, gu, p0, r, i * SW, SW, act);
      }
      if (diag) {
#pragma unroll
        for (int p = 0; p < kP; ++p)
          if (act && p0 + 16 * p + r == i) {  // X_ii and the unpruned (X.X)_ii
            s.d1[i] = (double)xv[t][p];
            s.d2[i] = (double)acc[p][t];
          }
      }
    }
    // The block's norm terms: lane 4 g + p sums row g's 16 columns of tile p
    // in registers (tree levels 1-4), then levels 5 and 6 join the four tiles
    // across the lane quad.
    wave_sync();
    {
      const int g = lane >> 2, p = lane & 3;
      const double *src = sq + g * kWave + 16 * p;
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = src[u];
#pragma unroll
      for (int w = 1; w < 16; w <<= 1)
#pragma unroll
        for (int u = 0; u < 16; u += 2 * w) v[u] = v[u] + v[u + w];
      double tb = v[0];
      tb = tb + dpp<0xb1>(tb);
      tb = tb + dpp<0x4e>(tb);
      if (p == 0) {
        // block b = p0 / 64 enters row g's pairwise tree over all aligned
        // blocks (those outside the window are +0, and x + 0 == x for the
        // sums of squares here): as a right child it joins its left sibling
        // -- on the stack if that subtree holds a window block, else +0 --
        // and climbs; as a left child it waits on the stack
        int node = p0 >> 6, lvl = 0;
        while (node & 1) {
          if ((node << lvl) > b_first) tb = stk[g * kLev + lvl] + tb;
          pend &= ~(1u << lvl);
          node >>= 1;
          ++lvl;
        }
        stk[g * kLev + lvl] = tb;
        pend |= 1u << lvl;
      }
    }
    wave_sync();
  }
  wave_sync();

  // Norm row term: the pending left subtrees, each joined to everything right
  // of it (the lower levels; their missing right parts are +0)
  {
    const int g = lane >> 2;
    double e = 0.0;
    bool any = false;
    for (int l = 0; l < kLev; ++l)
      if ((pend >> l) & 1u) {
        const double v = stk[g * kLev + l];
        e = any ? v + e : v;
        any = true;
      }
    if ((lane & 3) == 0 && g < nrows) s.e[i0 + g] = e;
  }
  if (r == 0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int rr = Mfma<T>::row(q, t);
      if (rr >= nrows) continue;
      const int i = i0 + rr;
      const int ylen = ry[t].length(), ulen = ru[t].length();
      SY.base[i] = ylen ? ry[t].first : 0;
      SY.len[i] = ylen;
      if (WITH_U) {
        SU.base[i] = ulen ? ru[t].first : 0;
        SU.len[i] = ulen;
      }
      s.wy[i] = ry[t].count;
      s.wu[i] = ru[t].count;
      if (s.ly) s.ly[i] = ylen;
      if (s.lu) s.lu[i] = ulen;
      if (i < wlo || i >= wlo + nblk * kWave) {  // column i never swept
        s.d1[i] = 0.0;
        s.d2[i] = 0.0;
      }
    }
  }
}

template <typename T, bool WITH_U>
__global__ __launch_bounds__(256) void k_x2_band16(int N, SpanRot3<T> spans, const SP2State *st, T tau, StepScratch s,
                                                   int32_t *fallback)
{
  __shared__ double stk_s[kWpb][kR * kLev];
  __shared__ double sq_s[kWpb][kR * kWave];
  __shared__ int2 meta_s[kWpb][kMeta];
  int cur = 0;
  bool once = false;
  if (st) {
    if (st->stop) return;
    cur = st->cur;
    once = st->once != 0;
  }
  const int w = uni(threadIdx.x >> 6);
  const int grp = xcd_block(blockIdx.x, gridDim.x) * kWpb + w;
  const int i0 = grp * kR;
  if (i0 >= N) return;
  const int cy = cur == 2 ? 0 : cur + 1, cu = cur == 0 ? 2 : cur - 1;
  rows16<T, false, WITH_U>(N, i0, min(kR, N - i0), spans.b[cur], spans.b[cy], spans.b[cu], tau, once, s, stk_s[w],
                           sq_s[w], meta_s[w], fallback);
}

// ---------------------------------------------------------------------------
// One whole SP2 iteration in one launch
// ---------------------------------------------------------------------------

// The SP2 iteration's product on the span form with its first reduction
// level: every workgroup computes its 64 rows as k_x2_band16 does, then
// reduces them -- the traces and the norm's row sums to one node of the
// perfect pairwise tree over all rows (the tree the separate reduction kernels
// form, so the sums keep their bits), the widths and counts to their maxima and
// totals -- and writes partial xb of nq = ceil(N / 64).
template <typename T>
__global__ __launch_bounds__(256) void k_x2_band16_part(int N, SpanRot3<T> spans, const SP2State *st, T tau,
                                                        StepScratch s)
{
  __shared__ double stk_s[kWpb][kR * kLev];
  __shared__ double sq_s[kWpb][kR * kWave];
  __shared__ int2 meta_s[kWpb][kMeta];
  if (st->stop) return;  // the same in every workgroup
  const int cur = st->cur;
  const int w = uni(threadIdx.x >> 6), lane = lane_id();
  const int xb = xcd_block(blockIdx.x, gridDim.x);
  const int i0 = (xb * kWpb + w) * kR;
  if (i0 < N) {
    const int cy = cur == 2 ? 0 : cur + 1, cu = cur == 0 ? 2 : cur - 1;
    rows16<T>(N, i0, min(kR, N - i0), spans.b[cur], spans.b[cy], spans.b[cu], tau, st->once != 0, s, stk_s[w],
              sq_s[w], meta_s[w], s.flags);
  }
  __syncthreads();  // the row outputs of all four wavefronts are written
  if (w != 0) return;
  const int nq = s.nq;
  const int r = xb * (kWpb * kR) + lane;
  const bool in = r < N;
  const double a0 = wave_tree(in ? s.d1[r] : -0.0);
  const double a1 = wave_tree(in ? s.d2[r] : -0.0);
  const double a2 = wave_tree(in ? s.e[r] : -0.0);
  const int wy = in ? s.wy[r] : 0, wu = in ? s.wu[r] : 0;
  const int ly = in && s.ly ? s.ly[r] : 0, lu = in && s.lu ? s.lu[r] : 0;
  const int m0 = wmax(wy), m1 = wmax(wu), m2 = wmax(ly), m3 = wmax(lu);
  const long long ny = wsum(wy), nu = wsum(wu);
  if (lane == 0) {
    s.part[xb] = a0;
    s.part[nq + xb] = a1;
    s.part[2 * nq + xb] = a2;
    s.partw[xb] = m0;
    s.partw[nq + xb] = m1;
    s.partw[2 * nq + xb] = m2;
    s.partw[3 * nq + xb] = m3;
    s.partn[xb] = ny;
    s.partn[nq + xb] = nu;
  }
}

// Upper levels of the tree over the nq partials, then the SP2 decision, by one
// workgroup.  With `publish` (mapped pinned host memory, or null) the state
// after the decision is also written there -- or the unchanged state, when the
// solve had stopped before this launch.
__global__ __launch_bounds__(256) void k_step_final64(SP2State *st, SP2Cfg cfg, SP2Hist h, StepScratch s,
                                                      SP2State *publish)
{
  __shared__ double ws[3][kWpb];
  __shared__ int32_t wsi[4][kWpb];
  __shared__ long long wsl[2][kWpb];
  const int t = threadIdx.x, w = t >> 6, lane = lane_id();
  const int nq = s.nq;
  // every load is issued first (the partials are read whatever the state
  // says: they are in bounds, and unused when the solve has stopped)
  double v[3];
  if (nq <= 256) leaf_tree3<1>(s.part, nq, t, v);
  else if (nq <= 512) leaf_tree3<2>(s.part, nq, 2 * t, v);
  else if (nq <= 1024) leaf_tree3<4>(s.part, nq, 4 * t, v);
  else if (nq <= 2048) leaf_tree3<8>(s.part, nq, 8 * t, v);
  else if (nq <= 4096) leaf_tree3<16>(s.part, nq, 16 * t, v);
  else if (nq <= 8192) leaf_tree3<32>(s.part, nq, 32 * t, v);
  else leaf_tree3<64>(s.part, nq, 64 * t, v);
  int32_t mx[4] = {0, 0, 0, 0};
  long long sy = 0, su = 0;
  for (int b = t; b < nq; b += 256) {
    for (int c = 0; c < 4; ++c) mx[c] = max(mx[c], s.partw[c * nq + b]);
    sy += s.partn[b];
    su += s.partn[nq + b];
  }
  SP2State x;
  if (t == 0) x = *st;
  if (st->stop) {
    if (publish && t == 0) {
      *publish = x;
      __threadfence_system();
    }
    return;
  }
  for (int c = 0; c < 3; ++c) v[c] = wave_tree(v[c]);
  for (int c = 0; c < 4; ++c) mx[c] = wmax(mx[c]);
  sy = wsum(sy);
  su = wsum(su);
  if (lane == 0) {
    for (int c = 0; c < 3; ++c) ws[c][w] = v[c];
    for (int c = 0; c < 4; ++c) wsi[c][w] = mx[c];
    wsl[0][w] = sy;
    wsl[1][w] = su;
  }
  __syncthreads();
  if (t == 0) {
    for (int c = 0; c < 3; ++c) s.out[c] = (ws[c][0] + ws[c][1]) + (ws[c][2] + ws[c][3]);
    for (int c = 0; c < 4; ++c) s.outw[c] = max(max(wsi[c][0], wsi[c][1]), max(wsi[c][2], wsi[c][3]));
    s.outn[0] = wsl[0][0] + wsl[0][1] + wsl[0][2] + wsl[0][3];
    s.outn[1] = wsl[1][0] + wsl[1][1] + wsl[1][2] + wsl[1][3];
    sp2dev::decide(&x, cfg, h, s);
    *st = x;
    if (publish) {
      *publish = x;
      __threadfence_system();
    }
  }
}

// Batched form: the instances' rows are stacked in one span matrix, instance m
// from row r0[m] (a multiple of 16), with its own local column numbers.  Group
// grp (16 rows) belongs to the instance of its first 8-row group; the wave
// works on that instance's rows as a matrix of its own, so every row, its
// column blocks and the norm's tree see exactly the coordinates of a single
// solve.  The instance's state selects the buffers, whether it still runs and
// its precision; the launch for one precision skips instances in the other.
template <typename T>
__device__ __forceinline__ SpanView<T> rows_from(SpanView<T> v, int r0)
{
  v.val += (size_t)r0 * v.SW;
  v.base += r0;
  v.len += r0;
  return v;
}

template <typename T, bool SYMA>
__global__ __launch_bounds__(256) void k_x2_band16_batch(int ngroups, SpanRot3<T> spans, const int32_t *grp_inst,
                                                         const int32_t *inst_r0, const int32_t *inst_rows,
                                                         const SP2State *states, int32_t phase32, const T *taus,
                                                         const StepScratch *ss, int32_t *flags)
{
  __shared__ double stk_s[kWpb][kR * kLev];
  __shared__ double sq_s[kWpb][kR * kWave];
  __shared__ int2 meta_s[kWpb][kMeta];
  const int w = uni(threadIdx.x >> 6);
  const int grp = xcd_block(blockIdx.x, gridDim.x) * kWpb + w;
  if (grp >= ngroups) return;
  const int m = uni(grp_inst[grp * (kR / kGroupRows)]);
  const SP2State *st = states + m;
  if (st->stop || st->phase32 != phase32) return;
  const int cur = uni(st->cur);
  const int cy = cur == 2 ? 0 : cur + 1, cu = cur == 0 ? 2 : cur - 1;
  const int r0 = uni(inst_r0[m]), n = uni(inst_rows[m]);
  const int i0 = grp * kR - r0;
  if (i0 >= n) return;  // alignment rows after the instance's last row
  rows16<T, SYMA>(n, i0, min(kR, n - i0), rows_from(spans.b[cur], r0), rows_from(spans.b[cy], r0),
            rows_from(spans.b[cu], r0), taus[m], st->once != 0, ss[m], stk_s[w], sq_s[w], meta_s[w], flags + m);
}

}  // namespace

bool x2_band16_fits(int N, int SW, int elem_bytes) { return (int64_t)N * SW * elem_bytes < ((int64_t)1 << 31); }

template <typename T>
hipError_t launch_x2_band16(int N, SpanRot3<T> spans, const SP2State *st, T tau, const StepScratch &s,
                            int32_t *fallback, hipStream_t stream, bool with_u)
{
  const int groups = (N + kR - 1) / kR;
  const dim3 grid((groups + kWpb - 1) / kWpb), block(kWpb * kWave);
  if (with_u)
    hipLaunchKernelGGL((k_x2_band16<T, true>), grid, block, 0, stream, N, spans, st, tau, s, fallback);
  else
    hipLaunchKernelGGL((k_x2_band16<T, false>), grid, block, 0, stream, N, spans, st, tau, s, fallback);
  return hipGetLastError();
}
template hipError_t launch_x2_band16<double>(int, SpanRot3<double>, const SP2State *, double, const StepScratch &,
                                             int32_t *, hipStream_t, bool);
template hipError_t launch_x2_band16<float>(int, SpanRot3<float>, const SP2State *, float, const StepScratch &,
                                            int32_t *, hipStream_t, bool);

template <typename T>
hipError_t launch_x2_band16_part(int N, SpanRot3<T> spans, const SP2State *st, T tau, const StepScratch &s,
                                 hipStream_t stream)
{
  const int groups = (N + kR - 1) / kR;
  const int blocks = (groups + kWpb - 1) / kWpb;
  if (blocks != s.nq || s.nq > 16384) return hipErrorInvalidValue;  // partials sized for N rows
  hipLaunchKernelGGL(k_x2_band16_part<T>, dim3(blocks), dim3(kWpb * kWave), 0, stream, N, spans, st, tau, s);
  return hipGetLastError();
}
template hipError_t launch_x2_band16_part<double>(int, SpanRot3<double>, const SP2State *, double,
                                                  const StepScratch &, hipStream_t);
template hipError_t launch_x2_band16_part<float>(int, SpanRot3<float>, const SP2State *, float, const StepScratch &,
                                                 hipStream_t);

hipError_t launch_step_final64(SP2State *st, const SP2Cfg &cfg, const SP2Hist &h, const StepScratch &s,
                               SP2State *publish, hipStream_t stream)
{
  if (s.nq > 16384) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_step_final64, dim3(1), dim3(kWpb * kWave), 0, stream, st, cfg, h, s, publish);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_x2_band16_batch(int ngroups16, SpanRot3<T> spans, const int32_t *grp_inst, const int32_t *inst_r0,
                                  const int32_t *inst_rows, const SP2State *states, int32_t phase32, const T *taus,
                                  const StepScratch *ss, int32_t *flags, bool sym, hipStream_t stream)
{
  static_assert(kR % kGroupRows == 0, "a 16-row group is a whole number of 8-row groups");
  const dim3 grid((ngroups16 + kWpb - 1) / kWpb), block(kWpb * kWave);
  if (sym)
    hipLaunchKernelGGL((k_x2_band16_batch<T, true>), grid, block, 0, stream, ngroups16, spans, grp_inst, inst_r0,
                       inst_rows, states, phase32, taus, ss, flags);
  else
    hipLaunchKernelGGL((k_x2_band16_batch<T, false>), grid, block, 0, stream, ngroups16, spans, grp_inst, inst_r0,
                       inst_rows, states, phase32, taus, ss, flags);
  return hipGetLastError();
}
template hipError_t launch_x2_band16_batch<double>(int, SpanRot3<double>, const int32_t *, const int32_t *,
                                                   const int32_t *, const SP2State *, int32_t, const double *,
                                                   const StepScratch *, int32_t *, bool, hipStream_t);
template hipError_t launch_x2_band16_batch<float>(int, SpanRot3<float>, const int32_t *, const int32_t *,
                                                  const int32_t *, const SP2State *, int32_t, const float *,
                                                  const StepScratch *, int32_t *, bool, hipStream_t);

}  // namespace ellsp2
