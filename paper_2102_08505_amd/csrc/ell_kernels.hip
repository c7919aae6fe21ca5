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
#include <algorithm>
#include <climits>
#include <cmath>

#include "ell_internal.h"
#include "sp2_decide.h"
#include "../../include/ellsp2.h"

namespace ellsp2 {
namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kWin = 512;        // accumulator window per wave (entries)
constexpr int kLev = 16;         // levels of a row's norm tree over aligned 64-column blocks (2^16 blocks)

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
__device__ __forceinline__ int rdlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float rdlane(float v, int l)
{
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double rdlane(double v, int l)
{
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

constexpr int kRowChunks = 4;  // row i held in registers when it has <= 256 entries
constexpr int kBatch = 8;      // rows k whose entries are loaded before their updates

// Running state of the ascending sweep over one output row.
struct SweepState {
  int cy, cu;     // kept X^2 entries, kept 2X - X^2 entries
  uint32_t pend;  // lane 0: bit l set when stk[l] holds a completed left subtree of 2^l blocks
};

// The norm's row term is the perfect pairwise tree over the row's column
// positions; every aligned 64-column block is one of its subtrees.  Blocks
// arrive in ascending order from the window's first block b_first on; block b
// (total t) enters the tree over all blocks, those outside the window being
// +0 (and x + 0 == x for these sums of squares): as a right child it joins its
// left sibling -- on the stack when that subtree holds a window block, else
// +0 -- and climbs; as a left child it waits on the stack.
__device__ __forceinline__ void push_block(double *stk, uint32_t &pend, const int b, const int b_first, double t)
{
  int node = b, lvl = 0;
  while (node & 1) {
    if ((node << lvl) > b_first) t = stk[lvl] + t;
    pend &= ~(1u << lvl);
    node >>= 1;
    ++lvl;
  }
  stk[lvl] = t;
  pend |= 1u << lvl;
}

// Sweep one accumulator window in ascending column order (the window starts
// on a multiple of 64 columns): compact the kept entries of X^2 (and of
// 2X - X^2), and reduce each aligned 64-column block of the norm's squared
// differences by the lane tree into the row's block tree (lane 0).  `once`:
// 2X - X^2 and the norm take the unpruned X^2 (one pruning per iteration);
// otherwise the pruned X^2.
template <typename T, bool WITH_U>
__device__ __forceinline__ void sweep_window(const int i, const int wlo, const int wlen, const T tau, const bool once,
                                             const T *acc, const T *xw, const int b_first, double *stk,
                                             const EllView<T> &Y, const EllView<T> &U, SweepState &st)
{
  const int lane = lane_id();
  for (int q0 = 0; q0 < wlen; q0 += kWave) {
    const int p = q0 + lane;
    const bool in = p < wlen;
    const int j = wlo + p;
    const T y = in ? acc[p] : T(0);
    const bool ky = in && absv(y) > tau;
    const T x = in ? xw[p] : T(0);
    const uint64_t my = __ballot(ky);
    if (ky) {
      const int pos = st.cy + lanes_below(my);
      if (pos < Y.M) {
        Y.idx[(size_t)i * Y.M + pos] = j;
        Y.val[(size_t)i * Y.M + pos] = y;
      }
    }
    st.cy += __popcll(my);
    const T ym = (ky || once) ? y : T(0);  // the X^2 value 2X - X^2 and the norm see
    if (WITH_U) {
      const T v = T(2) * x - ym;
      const bool ku = in && absv(v) > tau;
      const uint64_t mu = __ballot(ku);
      if (ku) {
        const int pos = st.cu + lanes_below(mu);
        if (pos < U.M) {
          U.idx[(size_t)i * U.M + pos] = j;
          U.val[(size_t)i * U.M + pos] = v;
        }
      }
      st.cu += __popcll(mu);
    }
    const double dd = (double)ym - (double)x;
    const double t = wave_tree(dd * dd);
    if (lane == 0) push_block(stk, st.pend, (wlo + q0) >> 6, b_first, t);
  }
}

// Norm row term (lane 0): the pending left subtrees, each joined to everything
// right of it (the lower levels; their missing right parts are +0).
__device__ __forceinline__ double finish_norm(const double *stk, const uint32_t pend)
{
  double e = 0.0;
  bool any = false;
  for (int l = 0; l < kLev; ++l)
    if ((pend >> l) & 1u) {
      const double v = stk[l];
      e = any ? v + e : v;
      any = true;
    }
  return e;
}

// Accumulate the products of rows k = row i's columns into the window
// [wlo, wlo + wlen): k ascending, the lanes over row k's entries.  Row i
// (columns kk, values aa, widths nkk) is held in registers, lane s of chunk c
// holding entry 64c + s; the entries of kBatch consecutive rows k are loaded
// before any of their updates, and the updates are applied in k order.
template <typename T>
__device__ __forceinline__ void accumulate_window(const int wi, const int wlo, const int wlen,
                                                  const int32_t *__restrict__ xidx,
                                                  const T *__restrict__ xval, const int M,
                                                  const int (&kk)[kRowChunks], const T (&aa)[kRowChunks],
                                                  const int (&nkk)[kRowChunks], T *acc)
{
  const int lane = lane_id();
#pragma unroll
  for (int c = 0; c < kRowChunks; ++c) {
    const int sbeg = c * kWave;
    if (sbeg >= wi) break;
    const int send = min(wi, sbeg + kWave);
    for (int s0 = sbeg; s0 < send; s0 += kBatch) {
      int kb[kBatch], nb[kBatch];
      T ab[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int s = s0 + u;
        const bool ok = s < send;
        kb[u] = ok ? rdlane(kk[c], s & 63) : 0;
        ab[u] = ok ? rdlane(aa[c], s & 63) : T(0);
        nb[u] = ok ? rdlane(nkk[c], s & 63) : 0;
      }
      int jj[kBatch][2];
      T vv[kBatch][2];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int32_t *ck = xidx + (size_t)kb[u] * M;
        const T *vk = xval + (size_t)kb[u] * M;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int t = lane + h * kWave;
          const bool ok = t < nb[u];
          jj[u][h] = ok ? ck[t] : -1;
          vv[u][h] = ok ? vk[t] : T(0);
        }
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int p = jj[u][h] - wlo;
          if ((unsigned)p < (unsigned)wlen) acc[p] = fmadd(ab[u], vv[u][h], acc[p]);
        }
        if (nb[u] > 2 * kWave) {  // rows k wider than 128: the rest, still before row k+1
          const int32_t *ck = xidx + (size_t)kb[u] * M;
          const T *vk = xval + (size_t)kb[u] * M;
          for (int t = lane + 2 * kWave; t < nb[u]; t += kWave) {
            const int p = ck[t] - wlo;
            if ((unsigned)p < (unsigned)wlen) acc[p] = fmadd(ab[u], vk[t], acc[p]);
          }
        }
      }
    }
  }
}

template <typename T, bool WITH_U>
__device__ void x2_row(const int i, const int32_t *__restrict__ xnnz, const int32_t *__restrict__ xidx,
                       const T *__restrict__ xval, const int M, EllView<T> Y, EllView<T> U, const T tau,
                       const bool once, T *acc, T *xw, double *stk, const StepScratch &s)
{
  const int lane = lane_id();
  const int wi = uniform_i(xnnz[i]);
  const int32_t *ci = xidx + (size_t)i * M;
  const T *vi = xval + (size_t)i * M;
  const bool regs = wi <= kWave * kRowChunks;

  // row i into registers (when it fits), the window bounds and X_ii
  int kk[kRowChunks], nkk[kRowChunks];
  T aa[kRowChunks];
#pragma unroll
  for (int c = 0; c < kRowChunks; ++c) {
    const int sl = c * kWave + lane;
    const bool ok = regs && sl < wi;
    kk[c] = ok ? ci[sl] : 0;
    aa[c] = ok ? vi[sl] : T(0);
  }
#pragma unroll
  for (int c = 0; c < kRowChunks; ++c) nkk[c] = (regs && c * kWave + lane < wi) ? xnnz[kk[c]] : 0;
  int lo = INT_MAX, hi = -1;
  double d1 = 0.0;
  bool has_diag = false;
  if (regs) {
#pragma unroll
    for (int c = 0; c < kRowChunks; ++c) {
      if (c * kWave + lane < wi) {
        const int k = kk[c];
        int f = k, l = k;
        if (nkk[c] > 0) {
          const int32_t *ck = xidx + (size_t)k * M;
          f = min(f, ck[0]);
          l = max(l, ck[nkk[c] - 1]);
        }
        lo = min(lo, f);
        hi = max(hi, l);
        if (k == i) {
          has_diag = true;
          d1 = (double)aa[c];
        }
      }
    }
  } else {
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
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  const uint64_t dm = __ballot(has_diag);
  if (dm) d1 = __shfl(d1, __builtin_ctzll(dm), kWave);

  SweepState st{0, 0, 0u};
  double d2 = 0.0;
  // windows start on multiples of 64 columns, so every 64-wide step of the
  // sweep is one aligned block of the norm's column tree
  const int lo_al = lo == INT_MAX ? lo : (lo & ~63);
  const int b_first = lo == INT_MAX ? 0 : (lo_al >> 6);
  for (int wlo = lo_al; wlo <= hi; wlo += kWin) {
    const int wlen = min(kWin, hi - wlo + 1);
    for (int p = lane; p < wlen; p += kWave) {
      acc[p] = T(0);
      xw[p] = T(0);
    }
    wave_sync();
    for (int s0 = 0; s0 < wi; s0 += kWave) {
      const int sl = s0 + lane;
      if (sl < wi) {
        const int p = ci[sl] - wlo;
        if ((unsigned)p < (unsigned)wlen) xw[p] = vi[sl];
      }
    }
    wave_sync();
    if (regs) {
      accumulate_window<T>(wi, wlo, wlen, xidx, xval, M, kk, aa, nkk, acc);
    } else {
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
    }
    wave_sync();
    if (i >= wlo && i < wlo + wlen) d2 = (double)acc[i - wlo];
    sweep_window<T, WITH_U>(i, wlo, wlen, tau, once, acc, xw, b_first, stk, Y, U, st);
  }
  const double ev = finish_norm(stk, st.pend);
  if (lane == 0) {
    Y.nnz[i] = min(st.cy, Y.M);
    s.wy[i] = st.cy;
    if (WITH_U) {
      U.nnz[i] = min(st.cu, U.M);
      s.wu[i] = st.cu;
    } else {
      s.wu[i] = 0;
    }
    s.d1[i] = d1;
    s.d2[i] = d2;
    s.e[i] = ev;
  }
}

// Block b runs on XCD b % 8; give each XCD a contiguous range of row groups so
// that the rows k its waves share stay in that XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int nblocks)
{
  constexpr int kXcd = 8;
  const int per = nblocks / kXcd;            // full share of every XCD
  const int full = per * kXcd;
  if (b >= full) return b;                   // the tail keeps its order
  return (b % kXcd) * per + b / kXcd;
}

// rows: null (row = wave index), or a list of *nrows rows to compute.
template <typename T, bool WITH_U>
__global__ __launch_bounds__(256) void k_x2_step(int N, Rot3<T> bufs, const SP2State *st, T tau,
                                                 StepScratch s, const int32_t *rows, const int32_t *nrows)
{
  __shared__ T acc_s[kWavesPerBlock][kWin];
  __shared__ T xw_s[kWavesPerBlock][kWin];
  __shared__ double stk_s[kWavesPerBlock][kLev];
  int cur = 0;
  bool once = false;
  if (st) {
    if (st->stop) return;
    cur = st->cur;
    once = st->once != 0;
  }
  const int w = uniform_i(threadIdx.x >> 6);
  int i = xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + w;
  if (rows) {
    if (i >= *nrows) return;
    i = uniform_i(rows[i]);
  }
  if (i >= N) return;
  const EllView<T> X = bufs.b[cur];
  const EllView<T> Y = bufs.b[cur == 2 ? 0 : cur + 1];
  const EllView<T> U = bufs.b[cur == 0 ? 2 : cur - 1];
  x2_row<T, WITH_U>(i, X.nnz, X.idx, X.val, X.M, Y, U, tau, once, acc_s[w], xw_s[w], stk_s[w], s);
}

// --------------------------------------------------------------------------
// the same row product with a hashed accumulator
// --------------------------------------------------------------------------
// For rows whose products are few and spread over a wide column range (the
// window kernel would sweep every 64-column block of the range): the row's
// distinct columns -- those of the rows k it references and its own -- go
// into an open-addressing table in LDS, are sorted (bitonic), and each gets
// its accumulator slot; the products are then added with fma in ascending k as
// in the window kernel, and the sorted columns are swept 64 at a time.  The
// norm's tree over column positions is built from the aligned 64-column
// blocks that hold columns, in ascending order; a block that holds none is a
// +0 subtree (x + 0 == x for these sums of squares), so the blocks combine at
// their lowest common ancestors, with the same bits as the window kernel.
// Rows with more than kHashCols products go to a list for the window kernel.
constexpr int kHashSlots = 1024;  // table slots per wave (a power of two)
constexpr int kHashCols = 512;    // products (and so distinct columns) a row may have here

template <typename T>
struct HashArena {
  int32_t key[kHashSlots];  // column, or -1
  int32_t pos[kHashSlots];  // position of the slot's column in col
  int32_t col[kHashCols];   // the row's columns, ascending
  T acc[kHashCols];         // (X.X)_ij at those columns
  T xv[kHashCols];          // X_ij at those columns
  double blk[kWave];        // squared differences of one aligned 64-column block
  double sv[kLev + 1];      // the norm's stack of subtree sums ...
  int32_t sl[kLev + 1];     // ... and the level at which each joins its left neighbour
};

__device__ __forceinline__ int hash_slot(int j) { return (int)(((uint32_t)j * 2654435761u) >> 22); }

// inserts j; true if it was not there
__device__ __forceinline__ bool hash_insert(int32_t *key, int j)
{
  int h = hash_slot(j);
  for (;;) {
    int expect = -1;
    if (__hip_atomic_compare_exchange_strong(&key[h], &expect, j, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WAVEFRONT))
      return true;
    if (expect == j) return false;
    h = (h + 1) & (kHashSlots - 1);
  }
}
// slot of j, or -1 when j is not in the table
__device__ __forceinline__ int hash_find(const int32_t *key, int j)
{
  int h = hash_slot(j);
  for (;;) {
    const int k = key[h];
    if (k == j) return h;
    if (k < 0) return -1;
    h = (h + 1) & (kHashSlots - 1);
  }
}

// Block b (ascending, any gaps) with total t joins the norm's tree: stack
// entries whose lowest common ancestor with their left neighbour lies below
// the one of b with the previous block form complete subtrees and are summed
// (left + right) first.  Lane 0.
template <typename T>
__device__ __forceinline__ void push_lca(HashArena<T> &ar, int &depth, int &prev, const int b, const double t)
{
  const int L = depth ? 32 - __builtin_clz((unsigned)(prev ^ b)) : INT_MAX;
  while (depth >= 2 && ar.sl[depth - 1] < L) {
    ar.sv[depth - 2] = ar.sv[depth - 2] + ar.sv[depth - 1];
    --depth;
  }
  ar.sv[depth] = t;
  ar.sl[depth] = L;
  ++depth;
  prev = b;
}

template <typename T, bool WITH_U>
__global__ __launch_bounds__(256) void k_x2_hash(int N, Rot3<T> bufs, T tau, StepScratch s, int32_t *left,
                                                 int32_t *nleft)
{
  __shared__ HashArena<T> ar_s[kWavesPerBlock];
  const int w = uniform_i(threadIdx.x >> 6), lane = lane_id();
  const int i = xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + w;
  if (i >= N) return;
  HashArena<T> &ar = ar_s[w];
  const EllView<T> X = bufs.b[0], Y = bufs.b[1], U = bufs.b[2];
  const int M = X.M;
  const int wi = uniform_i(X.nnz[i]);
  const int32_t *ci = X.idx + (size_t)i * M;
  const T *vi = X.val + (size_t)i * M;

  // products of the row (an upper bound on its distinct columns with wi)
  int P = 0;
  for (int s0 = 0; s0 < wi; s0 += kWave) {
    const int sl = s0 + lane;
    if (sl < wi) P += X.nnz[ci[sl]];
  }
  for (int o = 32; o > 0; o >>= 1) P += __shfl_xor(P, o, kWave);
  if (uniform_i(P) + wi > kHashCols) {
    if (lane == 0) left[atomicAdd(nleft, 1)] = i;
    return;
  }

  // the set of columns
  for (int h = lane; h < kHashSlots; h += kWave) ar.key[h] = -1;
  wave_sync();
  int E = 0;
  for (int s0 = 0; s0 < wi; s0 += kWave) {
    const int sl = s0 + lane;
    const bool ins = sl < wi && hash_insert(ar.key, ci[sl]);
    E += __popcll(__ballot(ins));
  }
  for (int s1 = 0; s1 < wi; ++s1) {
    const int k = uniform_i(ci[s1]);
    const int nk = uniform_i(X.nnz[k]);
    const int32_t *ck = X.idx + (size_t)k * M;
    for (int t0 = 0; t0 < nk; t0 += kWave) {
      const int t = t0 + lane;
      const bool ins = t < nk && hash_insert(ar.key, ck[t]);
      E += __popcll(__ballot(ins));
    }
  }
  wave_sync();
  E = uniform_i(E);

  // sorted columns and their slots
  int E2 = 1;
  while (E2 < E) E2 <<= 1;
  {
    int base = 0;
    for (int h0 = 0; h0 < kHashSlots; h0 += kWave) {
      const int key = ar.key[h0 + lane];
      const uint64_t m = __ballot(key >= 0);
      if (key >= 0) ar.col[base + lanes_below(m)] = key;
      base += __popcll(m);
    }
    for (int q = E + lane; q < E2; q += kWave) ar.col[q] = INT_MAX;
    wave_sync();
  }
  for (int size = 2; size <= E2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int p = lane; p < E2 / 2; p += kWave) {
        const int lo = 2 * stride * (p / stride) + (p % stride), hi = lo + stride;
        const bool up = (lo & size) == 0;
        const int a = ar.col[lo], b = ar.col[hi];
        if ((a > b) == up) {
          ar.col[lo] = b;
          ar.col[hi] = a;
        }
      }
      wave_sync();
    }
  for (int q = lane; q < E; q += kWave) {
    ar.pos[hash_find(ar.key, ar.col[q])] = q;
    ar.acc[q] = T(0);
    ar.xv[q] = T(0);
  }
  wave_sync();

  // X's own row, then the products, k ascending (the columns of one row k are
  // distinct, so lanes never meet in a slot)
  double d1 = 0.0;
  bool has_diag = false;
  for (int s0 = 0; s0 < wi; s0 += kWave) {
    const int sl = s0 + lane;
    if (sl < wi) {
      const int c = ci[sl];
      ar.xv[ar.pos[hash_find(ar.key, c)]] = vi[sl];
      if (c == i) {
        has_diag = true;
        d1 = (double)vi[sl];
      }
    }
  }
  const uint64_t dm = __ballot(has_diag);
  if (dm) d1 = __shfl(d1, __builtin_ctzll(dm), kWave);
  wave_sync();
  for (int s1 = 0; s1 < wi; ++s1) {
    const int k = uniform_i(ci[s1]);
    const T a = vi[s1];
    const int nk = uniform_i(X.nnz[k]);
    const int32_t *ck = X.idx + (size_t)k * M;
    const T *vk = X.val + (size_t)k * M;
    for (int t = lane; t < nk; t += kWave) {
      const int q = ar.pos[hash_find(ar.key, ck[t])];
      ar.acc[q] = fmadd(a, vk[t], ar.acc[q]);
    }
    wave_sync();
  }
  double d2 = 0.0;
  {
    const int h = hash_find(ar.key, i);
    if (h >= 0) d2 = (double)ar.acc[ar.pos[h]];
  }

  // sweep the sorted columns
  int cy = 0, cu = 0;
  int depth = 0, prev = 0, cb = -1;
  ar.blk[lane] = 0.0;
  wave_sync();
  for (int q0 = 0; q0 < E; q0 += kWave) {
    const int q = q0 + lane;
    const bool in = q < E;
    const int j = in ? ar.col[q] : INT_MAX;
    const T y = in ? ar.acc[q] : T(0);
    const T x = in ? ar.xv[q] : T(0);
    const bool ky = in && absv(y) > tau;
    const uint64_t my = __ballot(ky);
    if (ky) {
      const int p = cy + lanes_below(my);
      if (p < Y.M) {
        Y.idx[(size_t)i * Y.M + p] = j;
        Y.val[(size_t)i * Y.M + p] = y;
      }
    }
    cy += __popcll(my);
    const T yk = ky ? y : T(0);
    if (WITH_U) {
      const T v = T(2) * x - yk;
      const bool ku = in && absv(v) > tau;
      const uint64_t mu = __ballot(ku);
      if (ku) {
        const int p = cu + lanes_below(mu);
        if (p < U.M) {
          U.idx[(size_t)i * U.M + p] = j;
          U.val[(size_t)i * U.M + p] = v;
        }
      }
      cu += __popcll(mu);
    }
    const double dd = (double)yk - (double)x;
    const double sq = dd * dd;
    // the chunk's blocks in ascending order
    const int b = in ? (j >> 6) : INT_MAX;
    uint64_t todo = __ballot(in);
    while (todo) {
      const int bb = uniform_i(__shfl(b, (int)__builtin_ctzll(todo), kWave));
      if (bb != cb) {
        if (cb >= 0) {
          const double t = wave_tree(ar.blk[lane]);
          if (lane == 0) push_lca(ar, depth, prev, cb, t);
          wave_sync();
          ar.blk[lane] = 0.0;
          wave_sync();
        }
        cb = bb;
      }
      if (in && b == bb) ar.blk[j & 63] = sq;
      wave_sync();
      todo &= ~__ballot(in && b == bb);
    }
  }
  if (cb >= 0) {
    const double t = wave_tree(ar.blk[lane]);
    if (lane == 0) push_lca(ar, depth, prev, cb, t);
  }
  if (lane == 0) {
    while (depth >= 2) {
      ar.sv[depth - 2] = ar.sv[depth - 2] + ar.sv[depth - 1];
      --depth;
    }
    const double ev = depth ? ar.sv[0] : 0.0;
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

// --------------------------------------------------------------------------
// deterministic reductions of the step outputs
// --------------------------------------------------------------------------
// Partial sums of 1024 rows (block b of a matrix with N rows): perfect trees of
// d1, d2, e; maxima of the widths and interval lengths; nnz totals.
__device__ void step_partial(const int N, const StepScratch &s, const int b)
{
  __shared__ double ws[4];
  __shared__ int32_t wsi[4][4];
  __shared__ long long wsl[2][4];
  const int base = b * kRedBlock + threadIdx.x * 4;
  double a[3][4];
  int32_t mx[4] = {0, 0, 0, 0};
  long long sy = 0, su = 0;
  for (int q = 0; q < 4; ++q) {
    const int r = base + q;
    const bool in = r < N;
    a[0][q] = in ? s.d1[r] : -0.0;
    a[1][q] = in ? s.d2[r] : -0.0;
    a[2][q] = in ? s.e[r] : -0.0;
    if (in) {
      mx[0] = max(mx[0], s.wy[r]);
      mx[1] = max(mx[1], s.wu[r]);
      if (s.ly) mx[2] = max(mx[2], s.ly[r]);
      if (s.lu) mx[3] = max(mx[3], s.lu[r]);
      sy += s.wy[r];
      su += s.wu[r];
    }
  }
  double t[3];
  for (int c = 0; c < 3; ++c) t[c] = block_tree_1024(a[c][0], a[c][1], a[c][2], a[c][3], ws);
  for (int o = 32; o > 0; o >>= 1) {
    for (int c = 0; c < 4; ++c) mx[c] = max(mx[c], __shfl_xor(mx[c], o, kWave));
    sy += __shfl_xor(sy, o, kWave);
    su += __shfl_xor(su, o, kWave);
  }
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    for (int c = 0; c < 4; ++c) wsi[c][w] = mx[c];
    wsl[0][w] = sy;
    wsl[1][w] = su;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = 0; c < 3; ++c) s.part[c * s.nb + b] = t[c];
    for (int c = 0; c < 4; ++c)
      s.partw[c * s.nb + b] = max(max(wsi[c][0], wsi[c][1]), max(wsi[c][2], wsi[c][3]));
    s.partn[b] = wsl[0][0] + wsl[0][1] + wsl[0][2] + wsl[0][3];
    s.partn[s.nb + b] = wsl[1][0] + wsl[1][1] + wsl[1][2] + wsl[1][3];
  }
}

__global__ __launch_bounds__(256) void k_step_partial(int N, const SP2State *st, StepScratch s)
{
  if (st && st->stop) return;
  step_partial(N, s, blockIdx.x);
}

// Batched form: launch block b reduces block blk_local[b] of instance blk_inst[b],
// with that instance's row count, scratch view and state.
__global__ __launch_bounds__(256) void k_step_partial_batch(const int32_t *blk_inst, const int32_t *blk_local,
                                                            const int32_t *inst_rows, const StepScratch *ss,
                                                            const SP2State *states)
{
  const int m = blk_inst[blockIdx.x];
  if (states[m].stop) return;
  step_partial(inst_rows[m], ss[m], blk_local[blockIdx.x]);
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
  // maxima and integer totals: exact in any order, so spread over the block
  __shared__ int32_t wsi[4][4];
  __shared__ long long wsl[2][4];
  int32_t mx[4] = {0, 0, 0, 0};
  long long sy = 0, su = 0;
  for (int b = threadIdx.x; b < s.nb; b += 256) {
    for (int c = 0; c < 4; ++c) mx[c] = max(mx[c], s.partw[c * s.nb + b]);
    sy += s.partn[b];
    su += s.partn[s.nb + b];
  }
  for (int o = 32; o > 0; o >>= 1) {
    for (int c = 0; c < 4; ++c) mx[c] = max(mx[c], __shfl_xor(mx[c], o, kWave));
    sy += __shfl_xor(sy, o, kWave);
    su += __shfl_xor(su, o, kWave);
  }
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    for (int c = 0; c < 4; ++c) wsi[c][w] = mx[c];
    wsl[0][w] = sy;
    wsl[1][w] = su;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = 0; c < 4; ++c) s.outw[c] = max(max(wsi[c][0], wsi[c][1]), max(wsi[c][2], wsi[c][3]));
    s.outn[0] = wsl[0][0] + wsl[0][1] + wsl[0][2] + wsl[0][3];
    s.outn[1] = wsl[1][0] + wsl[1][1] + wsl[1][2] + wsl[1][3];
  }
}

__global__ __launch_bounds__(256) void k_step_final(SP2State *st, SP2Cfg cfg, SP2Hist h, StepScratch s)
{
  __shared__ double ws[4];
  if (st && st->stop) return;
  final_reduce(s, ws);
  __syncthreads();
  if (st && threadIdx.x == 0) sp2dev::decide(st, cfg, h, s);
}

// Batched form: block m finishes the reductions of instance m and takes its decision.
__global__ __launch_bounds__(256) void k_step_final_batch(SP2State *states, const SP2Cfg *cfgs, const SP2Hist *hists,
                                                          const StepScratch *ss)
{
  __shared__ double ws[4];
  const int m = blockIdx.x;
  if (states[m].stop) return;
  final_reduce(ss[m], ws);
  __syncthreads();
  if (threadIdx.x == 0) sp2dev::decide(&states[m], cfgs[m], hists[m], ss[m]);
}

// --------------------------------------------------------------------------
// initialisation: Gershgorin bounds and X0
// --------------------------------------------------------------------------

// One wavefront per kGershRows consecutive rows (rows strided over the grid).
// The rows' entries are staged through LDS kGershCols columns at a time, loaded
// coalesced (consecutive rows are contiguous in the ELLPACK arrays) and all in
// flight together before the first is stored; then lane
// t < kGershRows passes row i0 + t's staged entries in ascending j to one
// running sum r = r + |H_ij| (j != i), so the rows' serial sums run side by
// side.  Each workgroup writes the min / max of its rows' H_ii - r_i and
// H_ii + r_i (min and max are exact in any order).
constexpr int kGershCols = 136;  // 26 KiB of LDS; a 129-entry band row in one pass
constexpr int kGershStride = kGershCols + 1;  // LDS row stride: the summing lanes hit distinct banks
constexpr int kGershLoads = kGershRows * kGershCols / kWave;  // staged entries per lane and pass
static_assert(kGershRows * kGershCols % kWave == 0, "whole loads per lane");
// One group of rows i0 .. i0 + kGershRows - 1 (cut at N): lo / hi take the
// min / max of H_ii - r_i and H_ii + r_i, bad whether a stored value is not
// finite.  sv, sj: the wavefront's LDS staging.
__device__ __forceinline__ void gersh_group(int N, const EllView<double> &H, int i0, double *sv, int32_t *sj,
                                            double &lo, double &hi, bool &bad)
{
  const int lane = threadIdx.x;
  const int rows = min(kGershRows, N - i0);
  const int i = i0 + lane;
  const int n = lane < rows ? H.nnz[i] : 0;
  int nmax = n;
  for (int o = kWave / 2; o > 0; o >>= 1) nmax = max(nmax, __shfl_xor(nmax, o, kWave));
  double r = 0.0, hii = 0.0;
  for (int q0 = 0; q0 < nmax; q0 += kGershCols) {
    int jj[kGershLoads];
    double hh[kGershLoads];
#pragma unroll
    for (int k = 0; k < kGershLoads; ++k) {
      const int e = k * kWave + lane, t = e / kGershCols, q = q0 + e % kGershCols;
      const bool in = t < rows && q < __shfl(n, t, kWave);  // a stored entry of row i0 + t
      jj[k] = in ? H.idx[(size_t)(i0 + t) * H.M + q] : 0;
      hh[k] = in ? H.val[(size_t)(i0 + t) * H.M + q] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kGershLoads; ++k) {
      const int e = k * kWave + lane, t = e / kGershCols;
      sj[t * kGershStride + e % kGershCols] = jj[k];
      sv[t * kGershStride + e % kGershCols] = hh[k];
    }
    __syncthreads();
    const int cnt = min(kGershCols, n - q0);  // <= 0 past the row's end and for lanes >= rows
    // eight staged entries read before they are added in order, so that the
    // LDS latency is paid once per eight
    int c = 0;
    for (; c + 8 <= cnt; c += 8) {
      double hv[8];
      int jv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        hv[u] = sv[lane * kGershStride + c + u];
        jv[u] = sj[lane * kGershStride + c + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        bad = bad || !isfinite(hv[u]);
        if (jv[u] == i) hii = hv[u];
        else r = r + fabs(hv[u]);
      }
    }
    for (; c < cnt; ++c) {
      const double h = sv[lane * kGershStride + c];
      bad = bad || !isfinite(h);
      if (sj[lane * kGershStride + c] == i) hii = h;
      else r = r + fabs(h);
    }
    __syncthreads();
  }
  if (lane < rows) {
    lo = fmin(lo, hii - r);
    hi = fmax(hi, hii + r);
  }
}

// the wavefront's min / max to out_lo / out_hi, and flags |= 2 if bad
__device__ __forceinline__ void gersh_out(double lo, double hi, bool bad, double *out_lo, double *out_hi,
                                          int32_t *flags)
{
  for (int o = kWave / 2; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, kWave));
    hi = fmax(hi, __shfl_xor(hi, o, kWave));
  }
  if (__ballot(bad) && threadIdx.x == 0) atomicOr(flags, 2);
  if (threadIdx.x == 0) {
    *out_lo = lo;
    *out_hi = hi;
  }
}

__global__ __launch_bounds__(kWave) void k_gersh_rows(int N, EllView<double> H, double *plo, double *phi,
                                                      int32_t *flags)
{
  __shared__ double sv[kGershRows * kGershStride];
  __shared__ int32_t sj[kGershRows * kGershStride];
  double lo = INFINITY, hi = -INFINITY;
  bool bad = false;
  for (int i0 = blockIdx.x * kGershRows; i0 < N; i0 += gridDim.x * kGershRows) gersh_group(N, H, i0, sv, sj, lo, hi, bad);
  gersh_out(lo, hi, bad, plo + blockIdx.x, phi + blockIdx.x, flags);
}

// Instance of a multi-instance launch whose workgroups start at w0 (the
// instances in ascending w0; ws: their w0 in a separate array for the search).
__device__ __forceinline__ int inst_of(const int32_t *ws, int n, int w)
{
  int lo = 0, hi = n - 1;  // the last instance with ws[m] <= w
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ws[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Gershgorin over many matrices in one launch: one wavefront per group of
// kGershRows rows of one of them (workgroup b of instance m: rows 16 (b -
// w0[m]) .., strided by 16 nw[m] as in the single launch); the partial of
// workgroup b goes to plo[b], phi[b].
__global__ __launch_bounds__(kWave) void k_gersh_multi(const InitInst *in, const int32_t *ws, int n, double *plo,
                                                       double *phi, int32_t *flags)
{
  __shared__ double sv[kGershRows * kGershStride];
  __shared__ int32_t sj[kGershRows * kGershStride];
  const int m = inst_of(ws, n, blockIdx.x);
  const InitInst I = in[m];
  double lo = INFINITY, hi = -INFINITY;
  bool bad = false;
  for (int i0 = (blockIdx.x - I.w0) * kGershRows; i0 < I.N; i0 += I.nw * kGershRows)
    gersh_group(I.N, I.H, i0, sv, sj, lo, hi, bad);
  gersh_out(lo, hi, bad, plo + blockIdx.x, phi + blockIdx.x, flags + m);
}

// one workgroup per instance: min / max over its partials [w0, w0 + nw)
__global__ __launch_bounds__(256) void k_gersh_final_multi(const InitInst *in, const double *plo, const double *phi,
                                                           double *out)
{
  __shared__ double slo[256], shi[256];
  const InitInst I = in[blockIdx.x];
  double lo = INFINITY, hi = -INFINITY;
  for (int b = threadIdx.x; b < I.nw; b += 256) {
    lo = fmin(lo, plo[I.w0 + b]);
    hi = fmax(hi, phi[I.w0 + b]);
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
    out[2 * blockIdx.x] = slo[0];
    out[2 * blockIdx.x + 1] = shi[0];
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

// X0 = (emax I - H) inv, pruned, one wavefront per row (rows strided over at
// most kInitBlocks workgroups): the entries of row i in ascending column order,
// with the diagonal entry (emax - 0) inv put in its place when H stores none;
// kept values are compacted in order by ballot prefix counts, in one pass.  Per
// workgroup, an atomic max reports the widest row (skipped when the maximum
// already stored is as wide: after the first workgroups, nearly always) and,
// when `total` is given, an atomic add the count of kept entries.
// X0's row i of H into row ix of X (one wavefront; returns the kept count
// before the cut at X.M, the same on every lane).  One pass in ascending
// column order.  The diagonal H lacks, (emax - 0) inv, belongs between the
// entries with j < i and those with j > i; at the first entry with j >= i it
// is known whether H stores it (columns are sorted and unique), so the entries
// with j > i are placed one further when it is inserted, and the diagonal
// itself goes in at the end.
template <typename T>
__device__ __forceinline__ int x0_row(const EllView<double> &H, int i, const EllView<T> &X, int ix, double emax,
                                      double inv, T tau)
{
  const int lane = lane_id();
  const int n = uniform_i(H.nnz[i]);
  const int32_t *ci = H.idx + (size_t)i * H.M;
  const double *vi = H.val + (size_t)i * H.M;
  const T xd = (T)((emax - 0.0) * inv);
  int c = 0;       // kept entries of H so far
  int c_lt = -1;   // kept entries with j < i (once known)
  bool ins = false;
  for (int q0 = 0; q0 < n; q0 += kWave) {
    const int q = q0 + lane;
    const bool in = q < n;
    const int j = in ? ci[q] : INT_MAX;
    const double h = in ? vi[q] : 0.0;
    const double x = (j == i) ? (emax - h) * inv : (-h) * inv;
    const T xt = (T)x;
    const bool keep = in && absv(xt) > tau;
    const uint64_t m = __ballot(keep);
    if (c_lt < 0) {
      const uint64_t mge = __ballot(in && j >= i);
      if (mge) {
        const int f = __builtin_ctzll(mge);  // the first entry at or past the diagonal column
        c_lt = c + __popcll(m & ((1ull << f) - 1ull));
        ins = __ballot(in && j == i) == 0 && absv(xd) > tau;
      }
    }
    const int pos = c + lanes_below(m) + (ins && j > i ? 1 : 0);
    if (keep && pos < X.M) {
      X.idx[(size_t)ix * X.M + pos] = j;
      X.val[(size_t)ix * X.M + pos] = xt;
    }
    c += __popcll(m);
  }
  if (c_lt < 0) {  // every entry lies before the diagonal column
    c_lt = c;
    ins = absv(xd) > tau;
  }
  if (ins) {
    if (lane == 0 && c_lt < X.M) {
      X.idx[(size_t)ix * X.M + c_lt] = i;
      X.val[(size_t)ix * X.M + c_lt] = xd;
    }
    ++c;
  }
  if (lane == 0) X.nnz[ix] = min(c, X.M);
  return c;
}

template <typename T>
__global__ __launch_bounds__(256) void k_x0(int N, EllView<double> H, EllView<T> X, const double *ee, double emax,
                                            double inv, T tau, int32_t *wmax, unsigned long long *total)
{
  if (ee) {  // the bounds from the Gershgorin kernel: inv = 1 / (emax - emin), correctly rounded as on the host
    emax = ee[1];
    inv = 1.0 / (ee[1] - ee[0]);
  }
  __shared__ int smax[kWavesPerBlock];
  __shared__ unsigned long long ssum[kWavesPerBlock];
  const int w = threadIdx.x >> 6, lane = lane_id();
  int cmax = 0;
  unsigned long long csum = 0;
  for (int i = uniform_i(blockIdx.x * kWavesPerBlock + w); i < N; i += gridDim.x * kWavesPerBlock) {
    const int c = x0_row<T>(H, i, X, i, emax, inv, tau);
    cmax = max(cmax, c);
    csum += (unsigned long long)c;
  }
  if (lane == 0) {
    smax[w] = cmax;
    ssum[w] = csum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int m = max(max(smax[0], smax[1]), max(smax[2], smax[3]));
    if (m > __hip_atomic_load(wmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(wmax, m);
    if (total) atomicAdd(total, ssum[0] + ssum[1] + ssum[2] + ssum[3]);
  }
}

// X0 of many matrices in one launch, one wavefront per packed row r: the
// instance whose rows r0 .. r0 + N - 1 hold r (rows between instances and
// instances of the other precision are left alone); rowc[r] = the kept count.
template <typename T>
__global__ __launch_bounds__(256) void k_x0_multi(const InitInst *in, const int32_t *rs, int n, int rows,
                                                  EllView<T> X, int32_t *rowc)
{
  const int r = uniform_i(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
  if (r >= rows) return;
  const int m = inst_of(rs, n, r);
  const InitInst I = in[m];
  if (r - I.r0 >= I.N || I.f32 != (sizeof(T) == 4 ? 1 : 0)) return;
  const int c = x0_row<T>(I.H, r - I.r0, X, r, I.emax, I.inv, (T)I.tau);
  if (lane_id() == 0) rowc[r] = c;
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

// Bitwise symmetry of an ELLPACK matrix, one wavefront per row (rows strided
// over the grid).  Each stored (i, j) above the diagonal (j > i) is looked up
// in row j -- first at the mirror slot, then by bisection -- and *flag |= 1
// when (j, i) is absent or holds other bits; *balance gains the number of
// entries above the diagonal minus the number below it.  The mirrors found
// are distinct entries below the diagonal (one per entry above it), so with a
// zero balance they are all of them: H is bitwise symmetric iff the flag stays
// clear and the balance is zero.  (Half the lookups of checking both sides.)
// row i of the check: this lane's entries of the row (lanes over its entries)
__device__ __forceinline__ void check_row(const EllView<double> &H, int i, bool &bad, long long &bal)
{
  const int lane = lane_id();
  const int n = H.nnz[i];
  for (int s = lane; s < n; s += kWave) {
    const int j = H.idx[(size_t)i * H.M + s];
    if (j < i) --bal;
    if (j <= i) continue;
    ++bal;
    const double v = H.val[(size_t)i * H.M + s];
    const int32_t *cj = H.idx + (size_t)j * H.M;
    // first the mirror slot, where (j, i) sits when rows i and j are bands of
    // the same width (a slot below the capacity: in bounds whatever it holds)
    const int pm = n - 1 - s;
    const int nj = H.nnz[j];
    if (pm < H.M && cj[pm] == i && pm < nj) {
      bad = bad || __double_as_longlong(H.val[(size_t)j * H.M + pm]) != __double_as_longlong(v);
      continue;
    }
    int lo = 0, hi = nj - 1;
    bool found = false;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int c = cj[mid];
      if (c == i) {
        found = __double_as_longlong(H.val[(size_t)j * H.M + mid]) == __double_as_longlong(v);
        break;
      }
      if (c < i) lo = mid + 1;
      else hi = mid - 1;
    }
    bad = bad || !found;
  }
}

// the workgroup's results: flag |= 1 if any lane saw a missing or unequal
// mirror, the balance gains the workgroup's sum (one atomic, when nonzero)
__device__ __forceinline__ void check_out(bool bad, long long bal, int32_t *flag, unsigned long long *balance)
{
  __shared__ long long sb[kWavesPerBlock];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  if (__ballot(bad) && lane == 0) atomicOr(flag, 1);
  for (int o = kWave / 2; o > 0; o >>= 1) bal += __shfl_xor(bal, o, kWave);
  if (lane == 0) sb[w] = bal;
  __syncthreads();
  if (threadIdx.x == 0) {
    const long long t = (sb[0] + sb[1]) + (sb[2] + sb[3]);
    if (t != 0) atomicAdd(balance, (unsigned long long)t);  // (two's complement: a sum of signed counts)
  }
}

__global__ __launch_bounds__(256) void k_check_symmetric(int N, EllView<double> H, int32_t *flag,
                                                         unsigned long long *balance)
{
  bool bad = false;
  long long bal = 0;  // this lane's entries above minus below the diagonal
  for (int i = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); i < N; i += gridDim.x * kWavesPerBlock)
    check_row(H, i, bad, bal);
  check_out(bad, bal, flag, balance);
}

// the check of many matrices in one launch: workgroup b of instance m takes
// rows 4 (b - w0[m]) .. + 3, one per wavefront; instance m's flag word is
// flag[4m], its balance the 64 bits at flag + 4m + 2
__global__ __launch_bounds__(256) void k_check_symmetric_multi(const InitInst *in, const int32_t *ws, int n,
                                                               int32_t *flag)
{
  const int m = inst_of(ws, n, blockIdx.x);
  const InitInst I = in[m];
  const int i = (blockIdx.x - I.w0) * kWavesPerBlock + (threadIdx.x >> 6);
  bool bad = false;
  long long bal = 0;
  if (i < I.N) check_row(I.H, i, bad, bal);
  check_out(bad, bal, flag + 4 * m, reinterpret_cast<unsigned long long *>(flag + 4 * m + 2));
}

// n words set to zero (a kernel rather than a memset node, so that a caller
// may record it in a graph)
__global__ __launch_bounds__(256) void k_zero_words(int n, int32_t *p)
{
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}

// every array of the list, in one launch (grid-stride over each)
__global__ __launch_bounds__(256) void k_zero_list(ZeroList z)
{
  for (int a = 0; a < z.count; ++a)
    for (int i = blockIdx.x * 256 + threadIdx.x; i < z.n[a]; i += gridDim.x * 256) z.p[a][i] = 0;
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

// One thread per row i of A: t = fma(A_ij, B_ji, t) over row i in ascending j,
// B_ji found by a binary search of row j of B (columns ascending).
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_trace_product_rows(int N, EllView<TA> A, EllView<TB> B, double *d)
{
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  double t = 0.0;
  const int n = A.nnz[i];
  for (int q = 0; q < n; ++q) {
    const int j = A.idx[(size_t)i * A.M + q];
    const int32_t *cj = B.idx + (size_t)j * B.M;
    int lo = 0, hi = B.nnz[j] - 1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int c = cj[mid];
      if (c == i) {
        t = __builtin_fma((double)A.val[(size_t)i * A.M + q], (double)B.val[(size_t)j * B.M + mid], t);
        break;
      }
      if (c < i) lo = mid + 1;
      else hi = mid - 1;
    }
  }
  d[i] = t;
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
  const int32_t *none = nullptr;
  if (with_u)
    hipLaunchKernelGGL((k_x2_step<T, true>), grid, block, 0, stream, N, bufs, st, tau, s, none, none);
  else
    hipLaunchKernelGGL((k_x2_step<T, false>), grid, block, 0, stream, N, bufs, st, tau, s, none, none);
  return hipGetLastError();
}
template hipError_t launch_x2_step<double>(int, Rot3<double>, const SP2State *, bool, double,
                                           const StepScratch &, hipStream_t);
template hipError_t launch_x2_step<float>(int, Rot3<float>, const SP2State *, bool, float,
                                          const StepScratch &, hipStream_t);

template <typename T>
hipError_t launch_x2_hash(int N, Rot3<T> bufs, bool with_u, T tau, const StepScratch &s, int32_t *left,
                          int32_t *nleft, hipStream_t stream)
{
  const dim3 grid((N + kWavesPerBlock - 1) / kWavesPerBlock), block(256);
  hipError_t e = launch_zero_words(1, nleft, stream);
  if (e != hipSuccess) return e;
  if (with_u)
    hipLaunchKernelGGL((k_x2_hash<T, true>), grid, block, 0, stream, N, bufs, tau, s, left, nleft);
  else
    hipLaunchKernelGGL((k_x2_hash<T, false>), grid, block, 0, stream, N, bufs, tau, s, left, nleft);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the rows the table could not take, on the window kernel
  if (with_u)
    hipLaunchKernelGGL((k_x2_step<T, true>), grid, block, 0, stream, N, bufs, (const SP2State *)nullptr, tau, s,
                       (const int32_t *)left, (const int32_t *)nleft);
  else
    hipLaunchKernelGGL((k_x2_step<T, false>), grid, block, 0, stream, N, bufs, (const SP2State *)nullptr, tau, s,
                       (const int32_t *)left, (const int32_t *)nleft);
  return hipGetLastError();
}
template hipError_t launch_x2_hash<double>(int, Rot3<double>, bool, double, const StepScratch &, int32_t *,
                                           int32_t *, hipStream_t);
template hipError_t launch_x2_hash<float>(int, Rot3<float>, bool, float, const StepScratch &, int32_t *, int32_t *,
                                          hipStream_t);

hipError_t launch_reduce(int N, const SP2State *st, const StepScratch &s, hipStream_t stream)
{
  hipLaunchKernelGGL(k_step_partial, dim3(s.nb), dim3(256), 0, stream, N, st, s);
  return hipGetLastError();
}

hipError_t launch_decide(SP2State *st, SP2Cfg cfg, SP2Hist hist, const StepScratch &s, hipStream_t stream)
{
  hipLaunchKernelGGL(k_step_final, dim3(1), dim3(256), 0, stream, st, cfg, hist, s);
  return hipGetLastError();
}

hipError_t launch_reduce_batch(int nblocks, const int32_t *blk_inst, const int32_t *blk_local,
                               const int32_t *inst_rows, const StepScratch *ss, const SP2State *states,
                               hipStream_t stream)
{
  hipLaunchKernelGGL(k_step_partial_batch, dim3(nblocks), dim3(256), 0, stream, blk_inst, blk_local, inst_rows, ss,
                     states);
  return hipGetLastError();
}

hipError_t launch_decide_batch(int n, SP2State *states, const SP2Cfg *cfgs, const SP2Hist *hists,
                               const StepScratch *ss, hipStream_t stream)
{
  hipLaunchKernelGGL(k_step_final_batch, dim3(n), dim3(256), 0, stream, states, cfgs, hists, ss);
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
  const int nb = gersh_blocks(N);
  hipLaunchKernelGGL(k_gersh_rows, dim3(nb), dim3(kWave), 0, stream, N, H, rowlo, rowhi, flags);
  hipLaunchKernelGGL(k_gersh_final, dim3(1), dim3(256), 0, stream, nb, rowlo, rowhi, emin_emax);
  return hipGetLastError();
}

// X0's workgroups: one wavefront per row up to 32768 rows
static int x0_blocks(int N) { return std::min((N + kWavesPerBlock - 1) / kWavesPerBlock, 8192); }

template <typename T>
hipError_t launch_x0(int N, EllView<double> H, EllView<T> X, double emax, double inv, T tau, int32_t *wmax,
                     unsigned long long *total, hipStream_t stream)
{
  hipLaunchKernelGGL((k_x0<T>), dim3(x0_blocks(N)), dim3(256), 0, stream, N, H, X, (const double *)nullptr, emax,
                     inv, tau, wmax, total);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_x0(int N, EllView<double> H, EllView<T> X, const double *emin_emax, T tau, int32_t *wmax,
                     unsigned long long *total, hipStream_t stream)
{
  hipLaunchKernelGGL((k_x0<T>), dim3(x0_blocks(N)), dim3(256), 0, stream, N, H, X, emin_emax, 0.0, 0.0, tau, wmax,
                     total);
  return hipGetLastError();
}
template hipError_t launch_x0<double>(int, EllView<double>, EllView<double>, double, double, double,
                                      int32_t *, unsigned long long *, hipStream_t);
template hipError_t launch_x0<float>(int, EllView<double>, EllView<float>, double, double, float, int32_t *,
                                     unsigned long long *, hipStream_t);
template hipError_t launch_x0<double>(int, EllView<double>, EllView<double>, const double *, double, int32_t *,
                                      unsigned long long *, hipStream_t);
template hipError_t launch_x0<float>(int, EllView<double>, EllView<float>, const double *, float, int32_t *,
                                     unsigned long long *, hipStream_t);

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

hipError_t launch_check_symmetric(int N, EllView<double> H, int32_t *flag, unsigned long long *balance,
                                  hipStream_t stream)
{
  hipLaunchKernelGGL(k_check_symmetric, dim3(init_blocks(N)), dim3(256), 0, stream, N, H, flag, balance);
  return hipGetLastError();
}

hipError_t launch_gershgorin_multi(const InitInst *in, const int32_t *ws, int n, int nwork, double *plo,
                                   double *phi, double *out, int32_t *flags, hipStream_t stream)
{
  if (n <= 0 || nwork <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gersh_multi, dim3(nwork), dim3(kWave), 0, stream, in, ws, n, plo, phi, flags);
  hipLaunchKernelGGL(k_gersh_final_multi, dim3(n), dim3(256), 0, stream, in, plo, phi, out);
  return hipGetLastError();
}

hipError_t launch_check_symmetric_multi(const InitInst *in, const int32_t *ws, int n, int nwork, int32_t *flag,
                                        hipStream_t stream)
{
  if (n <= 0 || nwork <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_symmetric_multi, dim3(nwork), dim3(256), 0, stream, in, ws, n, flag);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_x0_multi(const InitInst *in, const int32_t *rs, int n, int rows, EllView<T> X, int32_t *rowc,
                           hipStream_t stream)
{
  if (n <= 0 || rows <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_x0_multi<T>), dim3((rows + kWavesPerBlock - 1) / kWavesPerBlock), dim3(256), 0, stream, in,
                     rs, n, rows, X, rowc);
  return hipGetLastError();
}
template hipError_t launch_x0_multi<double>(const InitInst *, const int32_t *, int, int, EllView<double>, int32_t *,
                                            hipStream_t);
template hipError_t launch_x0_multi<float>(const InitInst *, const int32_t *, int, int, EllView<float>, int32_t *,
                                           hipStream_t);

hipError_t launch_zero_words(int n, int32_t *p, hipStream_t stream)
{
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_words, dim3((n + 255) / 256), dim3(256), 0, stream, n, p);
  return hipGetLastError();
}

hipError_t launch_zero_list(const ZeroList &z, hipStream_t stream)
{
  int most = 0;
  for (int a = 0; a < z.count; ++a) most = std::max(most, z.n[a]);
  if (most <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_list, dim3(std::min((most + 255) / 256, 1024)), dim3(256), 0, stream, z);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_trace_rows(int N, EllView<T> A, double *d, hipStream_t stream)
{
  hipLaunchKernelGGL((k_trace_rows<T>), dim3((N + 255) / 256), dim3(256), 0, stream, N, A, d);
  return hipGetLastError();
}
template hipError_t launch_trace_rows<double>(int, EllView<double>, double *, hipStream_t);
template hipError_t launch_trace_rows<float>(int, EllView<float>, double *, hipStream_t);

template <typename TA, typename TB>
hipError_t launch_trace_product_rows(int N, EllView<TA> A, EllView<TB> B, double *d, hipStream_t stream)
{
  hipLaunchKernelGGL((k_trace_product_rows<TA, TB>), dim3((N + 255) / 256), dim3(256), 0, stream, N, A, B, d);
  return hipGetLastError();
}
template hipError_t launch_trace_product_rows<double, double>(int, EllView<double>, EllView<double>, double *,
                                                              hipStream_t);
template hipError_t launch_trace_product_rows<double, float>(int, EllView<double>, EllView<float>, double *,
                                                             hipStream_t);
template hipError_t launch_trace_product_rows<float, double>(int, EllView<float>, EllView<double>, double *,
                                                             hipStream_t);
template hipError_t launch_trace_product_rows<float, float>(int, EllView<float>, EllView<float>, double *,
                                                            hipStream_t);

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
