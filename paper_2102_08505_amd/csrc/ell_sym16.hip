// The SP2 iteration on the matrix cores for a bitwise symmetric span-form X,
// with the iteration's branch fixed before the product: one launch squares X
// (FP64 or FP32), writes only the iterate the branch selects (the pruned X^2,
// or the pruned 2X - X^2), reduces per 64-row workgroup the nodes of the
// pairwise trees of Tr X, the unpruned Tr X^2, the norm ||X^2 - X||_F^2, and
// Tr X' and Tr X'^2 of the iterate X' it wrote, and the workgroup that
// finishes last completes the trees and takes the decision: the
// "SP2 Loop X2", "SP2 Loop Norm" and "SP2 Loop Misc" steps of the paper's
// section "Performance Evaluation using an ExaSP2 Application", on the
// ELLPACK matrix-matrix multiply of its section "Performance Evaluation using
// System Matrices".
//
// Why the branch can be fixed first.  Iteration n chooses between X^2 and
// 2X - X^2 by comparing Tr X_n and the unpruned Tr X_n^2 with the
// occupation.  The row term (X_n^2)_ii is the chain of fused multiply-adds of
// X_ik X_ki over k ascending; when X_n is bitwise symmetric, X_ki = X_ik and
// the term is the ascending fma chain of the squares X_ik^2 over row i alone.
// The step that writes X_n forms that chain for every row it writes, so the
// decision after it already holds the branch of the next iteration.  An SP2
// trajectory from a symmetric H stays bitwise symmetric: X0 is; X^2 is (X^2_ij
// and X^2_ji sum the same products in the same k order); pruning and
// 2X - X^2 act entrywise.  Each step checks the prediction against the traces
// it computes from the product itself.
//
// Operand layout.  A's element X[i][k] is read as X[k][i], so one A load
// covers four rows k and sixteen consecutive columns (four 128-byte runs)
// instead of sixteen rows and four columns, which costs the memory pipeline
// four times as much.  The four 16x16 tiles of a 64-column block interleave
// their columns so that each lane's share of a row k is G = 16 / sizeof(T)
// consecutive columns, read with one 16-byte access: tile p, lane column r is
// column c0 + 16 G (p / G) + G r + p % G.  The span rows this kernel reads
// and writes therefore start on a multiple of G columns and hold a multiple
// of G positions (zeros at the ends), so a run of G columns is wholly inside
// or outside a row's interval.
//
// Every output entry is still the ascending-k fma chain of the row-by-row
// sparse product (the matrix instructions evaluate exactly that chain;
// positions outside an interval enter as zeros), so results are those of the
// oracle bit for bit.
#include <climits>

#include "band_common.h"
#include "ell_internal.h"
#include "sp2_decide.h"
#include "span16_common.h"

namespace ellsp2 {
namespace {

using namespace band;
using namespace span16;

constexpr int kR = 16;              // output rows per wave
constexpr int kP = 4;               // 16-column tiles per 64-column block
constexpr int kWpb = 4;             // waves per workgroup (64 rows)
constexpr int kKQ = 4;              // rows k whose intervals are held in registers: 64 kKQ
constexpr int kMeta = kKQ * kWave;  // entries of the wave's LDS table of row intervals
constexpr int kLev = 16;            // levels of the norm's block tree
constexpr int kSums = 5;            // Tr X, Tr X^2, eta^2, Tr X', Tr X'^2
constexpr int kSB = 1;              // 64-column blocks that share one pass over the rows k

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u32x4 ld16(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
  asm("" : "+v"(off));
  return __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
}
__device__ __forceinline__ void st16(__amdgpu_buffer_rsrc_t r, uint32_t off, u32x4 v)
{
  asm("" : "+v"(off));
  __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)off, 0, 0);
}

// G consecutive values of one 16-byte access
template <typename T>
struct Run {
  static constexpr int G = 16 / (int)sizeof(T);
  static constexpr int H = kP / G;  // 16-byte accesses per row per block
};
// (whole-vector casts: casting single elements of a 128-bit load result let
// the compiler narrow the load to its first dword)
typedef double f64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void unpack(u32x4 v, double *o)
{
  const f64x2 d = __builtin_bit_cast(f64x2, v);
  o[0] = d.x;
  o[1] = d.y;
}
__device__ __forceinline__ void unpack(u32x4 v, float *o)
{
  const f32x4 f = __builtin_bit_cast(f32x4, v);
  o[0] = f.x;
  o[1] = f.y;
  o[2] = f.z;
  o[3] = f.w;
}
__device__ __forceinline__ u32x4 pack(const double *o) { return __builtin_bit_cast(u32x4, f64x2{o[0], o[1]}); }
__device__ __forceinline__ u32x4 pack(const float *o)
{
  return __builtin_bit_cast(u32x4, f32x4{o[0], o[1], o[2], o[3]});
}

// first column of lane column r's run h in the block from column c0
template <typename T>
__device__ __forceinline__ int run_col(int c0, int h, int r)
{
  return c0 + 16 * Run<T>::G * h + Run<T>::G * r;
}

// Kept columns of one row of a block in column order (bit c of lo / hi:
// column p0 + c / p0 + 32 + c) from the four tiles' 16-bit row segments s[p]
// (bit r: tile p's lane column r).
__device__ __forceinline__ uint32_t spread2(uint32_t x)  // bit r -> bit 2r
{
  x = (x | (x << 8)) & 0x00ff00ffu;
  x = (x | (x << 4)) & 0x0f0f0f0fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}
__device__ __forceinline__ uint64_t spread4(uint64_t x)  // bit r -> bit 4r
{
  x = (x | (x << 24)) & 0x000000ff000000ffull;
  x = (x | (x << 12)) & 0x000f000f000f000full;
  x = (x | (x << 6)) & 0x0303030303030303ull;
  x = (x | (x << 3)) & 0x1111111111111111ull;
  return x;
}
__device__ __forceinline__ void row_cols(double, const uint32_t (&s)[kP], uint32_t &lo, uint32_t &hi)
{
  lo = spread2(s[0]) | spread2(s[1]) << 1;
  hi = spread2(s[2]) | spread2(s[3]) << 1;
}
__device__ __forceinline__ void row_cols(float, const uint32_t (&s)[kP], uint32_t &lo, uint32_t &hi)
{
  const uint64_t m = spread4(s[0]) | spread4(s[1]) << 1 | spread4(s[2]) << 2 | spread4(s[3]) << 3;
  lo = (uint32_t)m;
  hi = (uint32_t)(m >> 32);
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Accumulate kSB consecutive 64-column blocks (a superblock of 4 kSB
// tiles): acc[p] += X[i0 .. i0+15][k] X[k][tile p's columns] over
// k = klo .. khi, four k per step (a step past khi multiplies zeros); each A
// fragment feeds 4 kSB products, which keeps a step's matrix work above the
// latency of its loads.  A operand: lane (r, q) = (l % 16, l / 16) supplies X[k0 + q][i0 + r]
// (= X[i0 + r][k0 + q]); B operand of tile p: lane (r, q) supplies
// X[k0 + q][column of tile p, lane column r], G tiles from one 16-byte load.
// In FP64 the tiles of run h take part only in steps that meet that run's k
// range hlo[h] .. hhi[h] (its B operands are zeros elsewhere); in FP32 all
// four products issue.  Two operand sets alternate so that the loads of step
// k0 + 4 are in flight under the products of step k0.
template <typename T, bool LDS_META>
__device__ __forceinline__ void mma_block(const SpanView<T> &X, const __amdgpu_buffer_rsrc_t xr, const int2 *meta,
                                          const int kmin, const int kmax, const int klo, const int khi,
                                          const int (&hlo)[kSB * Run<T>::H], const int (&hhi)[kSB * Run<T>::H],
                                          const int p0, const int i0, typename Mfma<T>::acc (&acc)[kSB * kP])
{
  constexpr int G = Run<T>::G, H = kSB * Run<T>::H, NP = kSB * kP;
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
  auto load = [&](int k0, int2 m, T &a, T (&b)[NP]) {
    const int k = k0 + q;
    const int brow = k * SW - m.x;
    a = ld(xr, at<T>((unsigned)(i0 + r - m.x) < (unsigned)m.y, brow + i0 + r), T(0));
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int c = run_col<T>(p0, h, r);
      unpack(ld16(xr, at<T>((unsigned)(c - m.x) < (unsigned)m.y, brow + c)), b + G * h);
    }
  };
  auto mma = [&](int k0, T a, const T (&b)[NP]) {
#pragma unroll
    for (int h = 0; h < H; ++h)
      if (sizeof(T) == 4 || (k0 <= hhi[h] && k0 + 3 >= hlo[h])) {
#pragma unroll
        for (int g = 0; g < G; ++g) acc[G * h + g] = Mfma<T>::mma(a, b[G * h + g], acc[G * h + g]);
      }
  };
  const int nsteps = (khi - klo) / 4 + 1;
  T a0, b0[NP], a1, b1[NP];
  load(klo, interval(klo), a0, b0);
  int2 m1 = interval(klo + 4);
  int k0 = klo;
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

// Per-row results of a workgroup's 64 rows, reduced after its four waves.
struct RowOut {
  double s[kSums][kWpb * kR];
  int32_t wy[kWpb * kR];  // kept entries of the pruned X^2
  int32_t wo[kWpb * kR];  // kept entries of the written iterate
  int32_t lo[kWpb * kR];  // its interval length (a multiple of G)
};

// One wave: output rows i0 .. i0 + nrows - 1 (nrows <= 16).  X is read, the
// iterate the branch selects (UP: 2X - X^2, else X^2) is written to SO.  rw:
// the wave's 16 rows in the workgroup's RowOut.  `once`: 2X - X^2 and the
// norm take the unpruned X^2 (one pruning per iteration); otherwise the
// pruned X^2.
template <typename T, bool UP>
__device__ void rows16_sym(const int N, const int i0, const int nrows, const SpanView<T> X, const SpanView<T> SO,
                           const T tau, const bool once, double *stk, double *sq, int2 *meta, RowOut &ro,
                           const int rw)
{
  constexpr int G = Run<T>::G, H = Run<T>::H;
  const int lane = lane_id();
  const int r = lane & 15, q = lane >> 4;
  const int SW = X.SW;
  const int bytes = N * SW * (int)sizeof(T);  // < 2^31: the launcher takes this kernel only then
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(X.val, (short)0, bytes, kRawBufferFlags);
  const __amdgpu_buffer_rsrc_t orr = __builtin_amdgcn_make_buffer_rsrc(SO.val, (short)0, bytes, kRawBufferFlags);

  // interval of row r (lane l holds row l % 16)
  const int bA = r < nrows ? X.base[i0 + r] : 0;
  const int lA = r < nrows ? X.len[i0 + r] : 0;
  const int kmin = wmin(lA > 0 ? bA : INT_MAX);
  const int kmax = wmax(lA > 0 ? bA + lA - 1 : -1);
  if (kmax < 0) {
    // every row of the group is empty, and so is the iterate's
    if (q == 0 && r < nrows) {
      SO.base[i0 + r] = 0;
      SO.len[i0 + r] = 0;
    }
    if (q == 0) {
      for (int c = 0; c < kSums; ++c) ro.s[c][rw + r] = 0.0;
      ro.wy[rw + r] = 0;
      ro.wo[rw + r] = 0;
      ro.lo[rw + r] = 0;
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
  RowRun ry[4];  // the pruned X^2: its kept count only
  RowRun rx[4];  // the written iterate
  // X_ii, the unpruned (X.X)_ii and X'_ii, written by the lane that meets
  // column i (a column never swept holds no diagonal: they stay 0)
  if (q == 0) {
    ro.s[0][rw + r] = 0.0;
    ro.s[1][rw + r] = 0.0;
    ro.s[3][rw + r] = 0.0;
  }
  T chain = T(0);  // lanes 0..15: row lane's chain of squares of the iterate
  uint32_t pend = 0;  // the norm's pending subtrees of row lane / 4 (lanes 4 g)

  for (int pc = 0; pc < nblk; pc += kSB) {
    const int p0 = wlo + pc * kWave;  // the superblock's first column
    constexpr int HB = kSB * H;       // runs of the superblock
    // rows k whose interval meets each run's columns
    int hlo[HB], hhi[HB];
#pragma unroll
    for (int h = 0; h < HB; ++h) {
      hlo[h] = INT_MAX;
      hhi[h] = -1;
    }
    auto meet = [&](int kbase, int b, int l) {
#pragma unroll
      for (int h = 0; h < HB; ++h) {
        const int c0 = p0 + 16 * G * h;
        const uint64_t m = __ballot(l > 0 && b <= c0 + 16 * G - 1 && b + l - 1 >= c0);
        if (m) {
          hlo[h] = min(hlo[h], kbase + (int)__builtin_ctzll(m));
          hhi[h] = max(hhi[h], kbase + 63 - (int)__builtin_clzll(m));
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
    for (int h = 0; h < HB; ++h) {
      hlo[h] = uni(hlo[h]);
      hhi[h] = uni(hhi[h]);
      klo = min(klo, hlo[h]);
      khi = max(khi, hhi[h]);
    }
    typename Mfma<T>::acc acc[kSB * kP];
#pragma unroll
    for (int p = 0; p < kSB * kP; ++p) acc[p] = typename Mfma<T>::acc{T(0), T(0), T(0), T(0)};
    if (klo <= khi) {
      if (kfit) mma_block<T, true>(X, xr, meta, kmin, kmax, klo, khi, hlo, hhi, p0, i0, acc);
      else mma_block<T, false>(X, xr, meta, kmin, kmax, klo, khi, hlo, hhi, p0, i0, acc);
    }
#pragma unroll
    for (int sb = 0; sb < kSB; ++sb) {
      if (pc + sb >= nblk) break;  // (past the window: nothing to sweep)
      const int p0 = wlo + (pc + sb) * kWave;
      const bool diag = p0 <= i0 + kR - 1 && p0 + kWave - 1 >= i0;  // a diagonal entry lies in the block
      // Block p0 / 64 enters row g's pairwise norm tree over all aligned
      // blocks (outside the window: +0) with total tb: as a right child it
      // joins its left sibling and climbs; as a left child it waits on the
      // stack.  Lanes 4 g.
      auto enter = [&](double tb) {
        const int g = lane >> 2;
        int node = p0 >> 6, lvl = 0;
        while (node & 1) {
          if ((node << lvl) > b_first) tb = stk[g * kLev + lvl] + tb;
          pend &= ~(1u << lvl);
          node >>= 1;
          ++lvl;
        }
        stk[g * kLev + lvl] = tb;
        pend |= 1u << lvl;
      };
      // A block outside every row's interval of X (x = 0 there), without a
      // diagonal entry and with no entry of X^2 above tau keeps nothing and
      // writes nothing; when the norm takes the pruned X^2, each of its
      // squared differences is (+0 - +0)^2 = +0, so its norm node is +0, and
      // its terms of the iterate's chain of squares are fma(0, 0, c) = c.
      // Only that +0 node is entered, the sweep is skipped.  (Outside the
      // rows' intervals of the iterate, such blocks are most of a window's
      // ends: the unpruned product reaches twice as far as the pruned one.)
      if (!once && !diag) {
        const bool xin = r < nrows && lA > 0 && bA <= p0 + kWave - 1 && bA + lA - 1 >= p0;
        bool big = false;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int p = 0; p < kP; ++p) big |= Mfma<T>::row(q, t) < nrows && absv(acc[kP * sb + p][t]) > tau;
        if (__ballot(xin || big) == 0) {
          if ((lane & 3) == 0) enter(0.0);
          continue;
        }
      }
      // X at the block's output positions (for 2X - X^2 and the norm)
      T xv[4][kP];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int h = 0; h < H; ++h) {
          const int c = run_col<T>(p0, h, r);
          unpack(ld16(xr, at<T>((unsigned)(c - bC[t]) < (unsigned)lC[t], xrow[t] + c)), &xv[t][G * h]);
        }
      // sweep the block, four rows per set t (a row's 64 columns are the 16
      // lanes of its lane row q, G consecutive columns per run)
      T vks[4][kP];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int rr = Mfma<T>::row(q, t);
        const int i = i0 + rr;
        const bool act = rr < nrows;
        T vk[kP];
        bool ky[kP], kv[kP];
#pragma unroll
        for (int p = 0; p < kP; ++p) {
          const T y = acc[kP * sb + p][t], x = xv[t][p];
          ky[p] = act && absv(y) > tau;
          const T yk = ky[p] ? y : T(0);
          const T ym = once ? y : yk;  // the X^2 value 2X - X^2 and the norm see
          if (UP) {
            const T v = T(2) * x - ym;
            kv[p] = act && absv(v) > tau;
            vk[p] = kv[p] ? v : T(0);
          } else {  // the iterate is the pruned X^2 itself
            kv[p] = ky[p];
            vk[p] = yk;
          }
          const double d = (double)ym - (double)x;
          sq[rr * kWave + (run_col<T>(0, p / G, r) + p % G)] = d * d;
          vks[t][p] = vk[p];
        }
        uint32_t sy[kP], sv[kP];
        uint64_t anyv = 0;
#pragma unroll
        for (int p = 0; p < kP; ++p) {
          const uint64_t my = __ballot(ky[p]), mv = __ballot(kv[p]);
          sy[p] = seg16(my, q);
          sv[p] = seg16(mv, q);
          anyv |= mv;
        }
        ry[t].count += __popc(sy[0]) + __popc(sy[1]) + __popc(sy[2]) + __popc(sy[3]);
        // (a row quad that keeps nothing of the iterate in this block leaves
        // its row state as it is and writes nothing)
        if (anyv != 0) {
          uint32_t lo, hi;
          row_cols(T(0), sv, lo, hi);
          int gap;
          const int lw = rx[t].add(lo, hi, p0, gap);
          const int base = rx[t].first & ~(G - 1);
          const int row0 = i * SW;
#pragma unroll
          for (int h = 0; h < H; ++h) {
            const int c = run_col<T>(p0, h, r);
            const int o = c - base;
            st16(orr, at<T>(act && c <= lw && o >= 0 && o < SW, row0 + o), pack(&vk[G * h]));
          }
          // zeros for the runs after the row's last kept run of earlier blocks
          // up to this block (blocks that kept nothing)
          if (__ballot(gap < p0)) {
            const T z[G] = {};
            for (int c = ((gap + G - 1) & ~(G - 1)) + G * r; c < p0; c += 16 * G) {
              const int o = c - base;
              st16(orr, at<T>(act && o >= 0 && o < SW, row0 + o), pack(z));
            }
          }
        }
        if (diag) {
#pragma unroll
          for (int p = 0; p < kP; ++p)
            if (act && run_col<T>(p0, p / G, r) + p % G == i) {  // X_ii, the unpruned (X.X)_ii, X'_ii
              ro.s[0][rw + rr] = (double)xv[t][p];
              ro.s[1][rw + rr] = (double)acc[kP * sb + p][t];
              ro.s[3][rw + rr] = (double)vk[p];
            }
        }
      }
      // The block's norm terms: lane 4 g + j sums row g's 16 columns 16 j ..
      // 16 j + 15 in registers (tree levels 1-4), then levels 5 and 6 join the
      // four chunks across the lane quad.
      wave_sync();
      {
        const int g = lane >> 2, j = lane & 3;
        const double *src = sq + g * kWave + 16 * j;
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
        if (j == 0) enter(tb);
      }
      // The iterate's chain of squares: its values of the block to the same
      // table [row][column], then lane g < 16 runs row g's 64 columns in order.
      wave_sync();
      {
        T *vt = reinterpret_cast<T *>(sq);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int rr = Mfma<T>::row(q, t);
#pragma unroll
          for (int p = 0; p < kP; ++p) vt[rr * kWave + run_col<T>(0, p / G, r) + p % G] = vks[t][p];
        }
        wave_sync();
        if (lane < kR) {
          const T *row = vt + lane * kWave;
#pragma unroll 16
          for (int c = 0; c < kWave; ++c) chain = fma_t(row[c], row[c], chain);
        }
      }
      wave_sync();
    }
  }

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
    if ((lane & 3) == 0) ro.s[2][rw + g] = g < nrows ? e : 0.0;
  }
  if (lane < kR) ro.s[4][rw + lane] = lane < nrows ? (double)chain : 0.0;
  if (r == 0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int rr = Mfma<T>::row(q, t);
      const bool act = rr < nrows;
      const int i = i0 + rr;
      const int len = rx[t].length();
      const int base = len ? (rx[t].first & ~(G - 1)) : 0;
      const int alen = len ? (rx[t].last | (G - 1)) + 1 - base : 0;
      if (act) {
        SO.base[i] = base;
        SO.len[i] = alen;
      }
      ro.wy[rw + rr] = act ? ry[t].count : 0;
      ro.wo[rw + rr] = act ? rx[t].count : 0;
      ro.lo[rw + rr] = act ? alen : 0;
    }
  }
}

// Loads and stores of the partials that the last workgroup of a launch reads:
// coherent across the chip's L2 caches (agent scope), so that no release or
// acquire fence -- which would write back or invalidate a whole L2 -- is needed.
template <typename V>
__device__ __forceinline__ V cld(const V *p)
{
  return __hip_atomic_load(const_cast<V *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename V>
__device__ __forceinline__ void cst(V *p, V v)
{
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Perfect pairwise trees over the nq partials of sums c0 .. c0 + NS - 1, by
// one workgroup of 256: thread t holds the leaves [t L, t L + L) of each (L
// the smallest power of two with 256 L >= nq, nq <= 16384; leaves past nq are
// -0.0), then the trees over the threads.  The leaves past nq are loaded too
// (the partials are padded to 5 nq + 256 L), so that a thread's loads take
// one address.  Subtrees of up to 8 leaves issue every load before the first
// addition; larger ones sum their first half before loading the second, so
// that at most 8 leaves are live.
template <int L>
__device__ __forceinline__ double ctree(const double *p, int a, int n)
{
  if constexpr (L == 1) {
    const double x = cld(p + a);
    return a < n ? x : -0.0;
  } else if constexpr (L <= 8) {
    const double lo = ctree<L / 2>(p, a, n);
    return lo + ctree<L / 2>(p, a + L / 2, n);
  } else {
    double lo = ctree<L / 2>(p, a, n);
    asm volatile("" : "+v"(lo)::"memory");
    return lo + ctree<L / 2>(p, a + L / 2, n);
  }
}
template <int L, int NS>
__device__ __forceinline__ void leaves(const double *part, int nq, int t, double (&v)[NS])
{
  if constexpr (L <= 8) {
#pragma unroll
    for (int c = 0; c < NS; ++c) v[c] = ctree<L>(part + (size_t)c * nq, t * L, nq);
  } else {
#pragma unroll 1
    for (int c = 0; c < NS; ++c) v[c] = ctree<L>(part + (size_t)c * nq, t * L, nq);
  }
}
template <int NS>
__device__ __forceinline__ void thread_leaves(const double *part, int nq, int t, double (&v)[NS])
{
  if (nq <= 256) leaves<1>(part, nq, t, v);
  else if (nq <= 512) leaves<2>(part, nq, t, v);
  else if (nq <= 1024) leaves<4>(part, nq, t, v);
  else if (nq <= 2048) leaves<8>(part, nq, t, v);
  else if (nq <= 4096) leaves<16>(part, nq, t, v);
  else if (nq <= 8192) leaves<32>(part, nq, t, v);
  else leaves<64>(part, nq, t, v);
}
// the thread sums v into totals out[0 .. NS) (thread 0, which also keeps them
// in tot)
template <int NS>
__device__ __forceinline__ void tree_finish(double (&v)[NS], double *out, double *tot = nullptr)
{
  __shared__ double ws[NS][kWpb];
  const int t = threadIdx.x, w = t >> 6, lane = lane_id();
#pragma unroll
  for (int c = 0; c < NS; ++c) v[c] = wave_tree(v[c]);
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < NS; ++c) ws[c][w] = v[c];
  __syncthreads();
  if (t == 0)
    for (int c = 0; c < NS; ++c) {
      const double x = (ws[c][0] + ws[c][1]) + (ws[c][2] + ws[c][3]);
      out[c] = x;
      if (tot) tot[c] = x;
    }
}

// The SP2 iteration in one launch.  Each workgroup computes 64 rows, then
// reduces them -- the five sums to one node of the perfect pairwise tree over
// all rows (rows past N enter as -0.0, the exact additive identity), the
// widths to maxima, the kept counts to totals -- into partials xb of
// nq = ceil(N / 64), and takes a ticket once they are written; the workgroup
// that takes the last ticket builds the upper levels of the trees, takes the
// SP2 decision and returns the ticket counter to zero.  With `publish`
// (mapped pinned host memory, or null) the state afterwards is also written
// there -- or the unchanged state, when the solve had stopped before this
// launch.
template <typename T>
__global__ __launch_bounds__(256) void k_x2_sym_step(int N, SpanRot3<T> spans, SP2State *st, T tau, StepScratch s,
                                                     SP2Cfg cfg, SP2Hist h, SP2State *publish)
{
  __shared__ double stk_s[kWpb][kR * kLev];
  __shared__ double sq_s[kWpb][kR * kWave];
  __shared__ int2 meta_s[kWpb][kMeta];
  __shared__ RowOut ro;
  __shared__ int last_s;
  __shared__ int32_t wsi[3][kWpb];
  __shared__ long long wsl[2][kWpb];
  if (st->stop) {  // the same in every workgroup
    if (publish && blockIdx.x == 0 && threadIdx.x == 0) {
      *publish = *st;
      __threadfence_system();
    }
    return;
  }
  const int cur = st->cur;
  const bool up = st->up_next != 0;
  const int w = uni(threadIdx.x >> 6), lane = lane_id();
  const int xb = xcd_block(blockIdx.x, gridDim.x);
  const int i0 = (xb * kWpb + w) * kR;
  if (i0 < N) {
    // the iterate goes where the decision will find it: X^2 to slot cur + 1,
    // 2X - X^2 to slot cur + 2 (mod 3)
    const int co = up ? (cur == 0 ? 2 : cur - 1) : (cur == 2 ? 0 : cur + 1);
    const bool once = st->once != 0;
    if (up)
      rows16_sym<T, true>(N, i0, min(kR, N - i0), spans.b[cur], spans.b[co], tau, once, stk_s[w], sq_s[w],
                          meta_s[w], ro, w * kR);
    else
      rows16_sym<T, false>(N, i0, min(kR, N - i0), spans.b[cur], spans.b[co], tau, once, stk_s[w], sq_s[w],
                           meta_s[w], ro, w * kR);
  } else if (lane < kR) {
    for (int c = 0; c < kSums; ++c) ro.s[c][w * kR + lane] = -0.0;
    ro.wy[w * kR + lane] = 0;
    ro.wo[w * kR + lane] = 0;
    ro.lo[w * kR + lane] = 0;
  }
  __syncthreads();
  const int nq = s.nq;
  if (w == 0) {
    const bool in = xb * (kWpb * kR) + lane < N;
    double a[kSums];
#pragma unroll
    for (int c = 0; c < kSums; ++c) a[c] = wave_tree(in ? ro.s[c][lane] : -0.0);
    const int m0 = wmax(ro.wy[lane]), m1 = wmax(ro.wo[lane]), m2 = wmax(ro.lo[lane]);
    const long long ny = wsum(ro.wy[lane]), no = wsum(ro.wo[lane]);
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < kSums; ++c) cst(s.part + c * nq + xb, a[c]);
      cst(s.partw + xb, m0);
      cst(s.partw + nq + xb, m1);
      cst(s.partw + 2 * nq + xb, m2);
      cst(s.partn + xb, (int64_t)ny);
      cst(s.partn + nq + xb, (int64_t)no);
      // the partials are complete at agent scope before the ticket is taken
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      last_s = __hip_atomic_fetch_add(s.ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
    }
  }
  __syncthreads();
  if (!last_s) return;
  // the last workgroup: every other workgroup's partials are complete.  The
  // deciding thread loads the state (unchanged since the launch began) and
  // the norms of the products before this one under the partials' loads.
  const int t = threadIdx.x;
  SP2State x;
  sp2dev::SymOut o;
  if (t == 0) {
    x = *st;
    for (int q = 0; q < 3; ++q) {
      const int m = x.iter - 1 - q;
      o.prev[q] = m >= x.phase_start ? h.eta2[m] : 0.0;
    }
  }
  double v[kSums];
  thread_leaves(s.part, nq, t, v);
  int32_t mx[3] = {0, 0, 0};
  long long sy = 0, so = 0;
  for (int b = t; b < nq; b += 256) {
    for (int c = 0; c < 3; ++c) mx[c] = max(mx[c], cld(s.partw + c * nq + b));
    sy += cld(s.partn + b);
    so += cld(s.partn + nq + b);
  }
  for (int c = 0; c < 3; ++c) mx[c] = wmax(mx[c]);
  sy = wsum(sy);
  so = wsum(so);
  if (lane == 0) {
    for (int c = 0; c < 3; ++c) wsi[c][w] = mx[c];
    wsl[0][w] = sy;
    wsl[1][w] = so;
  }
  tree_finish(v, s.out, o.sum);  // (its barrier also covers wsi, wsl)
  if (t == 0) {
    for (int c = 0; c < 3; ++c) {
      o.w[c] = max(max(wsi[c][0], wsi[c][1]), max(wsi[c][2], wsi[c][3]));
      s.outw[c] = o.w[c];
    }
    for (int c = 0; c < 2; ++c) {
      o.n[c] = wsl[c][0] + wsl[c][1] + wsl[c][2] + wsl[c][3];
      s.outn[c] = o.n[c];
    }
    sp2dev::decide_sym(&x, cfg, h, o);
    *st = x;
    cst(s.ticket, 0u);
    if (publish) {
      *publish = x;
      __threadfence_system();
    }
  }
}

// The chain of squares of every row of a span matrix (the unpruned diagonal
// of its square when it is symmetric) and its diagonal, reduced per 64 rows
// like the step kernel's Tr X' and Tr X'^2: the first branch of a solve, and
// the branch after the precision switch.  One wave of 64 rows, lane l row
// 64 xb + l, reading its row G columns at a time in ascending order.
template <typename T>
__global__ __launch_bounds__(64) void k_sym_seed_part(int N, SpanRot3<T> spans, const SP2State *st, StepScratch s)
{
  constexpr int G = Run<T>::G;
  const SpanView<T> X = spans.b[st->cur];
  const int xb = blockIdx.x, lane = lane_id();
  const int i = xb * kWave + lane;
  double d1 = -0.0, d2 = -0.0;
  if (i < N) {
    const int SW = X.SW;
    const int bytes = N * SW * (int)sizeof(T);
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(X.val, (short)0, bytes, kRawBufferFlags);
    const int b = X.base[i], l = X.len[i];
    T c2 = T(0), dg = T(0);
    for (int p = 0; p < l; p += G) {
      T v[G];
      unpack(ld16(xr, at<T>(true, i * SW + p)), v);
#pragma unroll
      for (int g = 0; g < G; ++g) {
        c2 = fma_t(v[g], v[g], c2);
        if (b + p + g == i) dg = v[g];
      }
    }
    d1 = (double)dg;
    d2 = (double)c2;
  }
  d1 = wave_tree(d1);
  d2 = wave_tree(d2);
  if (lane == 0) {
    s.part[3 * s.nq + xb] = d1;
    s.part[4 * s.nq + xb] = d2;
  }
}

// The branch of the next product from the seed partials (Tr X, Tr X^2 of the
// current X), by one workgroup.
__global__ __launch_bounds__(256) void k_sym_seed_final(SP2State *st, SP2Cfg cfg, StepScratch s)
{
  double v[2];
  thread_leaves(s.part + 3 * (size_t)s.nq, s.nq, threadIdx.x, v);
  tree_finish(v, s.out + 3);
  if (threadIdx.x == 0) sp2dev::seed_sym(st, cfg, s.out[3], s.out[4]);
}

}  // namespace

template <typename T>
hipError_t launch_x2_sym_step(int N, SpanRot3<T> spans, SP2State *st, T tau, const StepScratch &s,
                              const SP2Cfg &cfg, const SP2Hist &h, SP2State *publish, hipStream_t stream)
{
  const int groups = (N + kR - 1) / kR;
  const int blocks = (groups + kWpb - 1) / kWpb;
  if (blocks != s.nq || s.nq > 16384 || !s.ticket) return hipErrorInvalidValue;  // partials sized for N rows
  hipLaunchKernelGGL(k_x2_sym_step<T>, dim3(blocks), dim3(kWpb * kWave), 0, stream, N, spans, st, tau, s, cfg, h,
                     publish);
  return hipGetLastError();
}
template hipError_t launch_x2_sym_step<double>(int, SpanRot3<double>, SP2State *, double, const StepScratch &,
                                               const SP2Cfg &, const SP2Hist &, SP2State *, hipStream_t);
template hipError_t launch_x2_sym_step<float>(int, SpanRot3<float>, SP2State *, float, const StepScratch &,
                                              const SP2Cfg &, const SP2Hist &, SP2State *, hipStream_t);

template <typename T>
hipError_t launch_sym_seed(int N, SpanRot3<T> spans, SP2State *st, const SP2Cfg &cfg, const StepScratch &s,
                           hipStream_t stream)
{
  const int nq = (N + kWave - 1) / kWave;
  if (nq != s.nq || s.nq > 16384) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sym_seed_part<T>, dim3(nq), dim3(kWave), 0, stream, N, spans, st, s);
  hipLaunchKernelGGL(k_sym_seed_final, dim3(1), dim3(kWpb * kWave), 0, stream, st, cfg, s);
  return hipGetLastError();
}
template hipError_t launch_sym_seed<double>(int, SpanRot3<double>, SP2State *, const SP2Cfg &, const StepScratch &,
                                            hipStream_t);
template hipError_t launch_sym_seed<float>(int, SpanRot3<float>, SP2State *, const SP2Cfg &, const StepScratch &,
                                           hipStream_t);

}  // namespace ellsp2
