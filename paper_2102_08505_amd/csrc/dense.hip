// Dense-block variant of the SP2 step on the matrix cores (gfx950).
//
// With a dense X the square X^2 is a plain dense contraction, so it runs on MFMA:
//  * BF16x3: X (float) is split once per step into hi = bf16(x) and
//    lo = bf16(x - hi) (round to nearest even), and X^2 is approximated by
//    hi.hi + hi.lo + lo.hi with float accumulation on v_mfma_f32_32x32x16_bf16
//    (the three-product split of Henry, Tang and Heinecke, ARITH 2019);
//  * FP64: v_mfma_f64_16x16x4_f64.
// Both GEMMs read their B operand from a transposed copy, so the values a lane
// feeds to one MFMA are contiguous along k.  After the product, one kernel per
// row forms 2X - X^2, both diagonals and the row term of the idempotency norm
// (pairwise tree over the N columns); the reductions and the device-side SP2
// decision are those of the sparse path (the SP2-Basic loop of the paper's
// section "Performance Evaluation using an ExaSP2 Application": an X^2 product,
// a matrix norm and the remaining update per iteration).  The paper has no
// dense variant; this one squares dense blocks on the matrix cores.
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/ellsp2.h"
#include "ell_internal.h"

namespace ellsp2 {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;
constexpr int kMaxDenseN = 32768;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// lane 0 receives the perfect pairwise tree over the 64 lanes
__device__ __forceinline__ double wave_tree(double v)
{
  for (int s = 1; s < kWave; s <<= 1) v = v + __shfl_down(v, s, kWave);
  return v;
}

// Operand selection: a fixed pair (x, y), or, during a solve, X = bufs[cur]
// and X^2 into bufs[(cur + 1) % 3] with cur read from the device state.
template <typename T>
struct DSel {
  const T *x;
  T *y;
  T *const *bufs;
  const SP2State *st;
};

template <typename T>
__device__ __forceinline__ bool resolve(const DSel<T> &s, const T *&x, T *&y)
{
  if (!s.st) {
    x = s.x;
    y = s.y;
    return true;
  }
  if (s.st->stop) return false;
  const int c = s.st->cur;
  x = s.bufs[c];
  y = s.bufs[c == 2 ? 0 : c + 1];
  return true;
}

// round to nearest even; bf16 held as its 16-bit pattern
__device__ __forceinline__ uint16_t bf16_bits(float x)
{
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) {
    if (u & 0x007fffffu) u |= 0x00400000u;
    return (uint16_t)(u >> 16);
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// hi/lo split of an N x N float matrix, row-major and transposed (32 x 32 tiles through LDS)
__global__ __launch_bounds__(256) void k_split(int N, DSel<float> sel, uint16_t *hi, uint16_t *lo, uint16_t *hiT,
                                               uint16_t *loT)
{
  __shared__ uint16_t th[32][33], tl[32][33];
  const float *X;
  float *unused;
  if (!resolve(sel, X, unused)) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + ty + 8 * q, c = c0 + tx;
    uint16_t h = 0, l = 0;
    if (r < N && c < N) {
      const float x = X[(size_t)r * N + c];
      h = bf16_bits(x);
      l = bf16_bits(x - bf16_val(h));
      hi[(size_t)r * N + c] = h;
      lo[(size_t)r * N + c] = l;
    }
    th[ty + 8 * q][tx] = h;
    tl[ty + 8 * q][tx] = l;
  }
  if (!hiT) return;  // (a symmetric X is its own transpose)
  __syncthreads();
  for (int q = 0; q < 4; ++q) {
    const int r = c0 + ty + 8 * q, c = r0 + tx;  // position in the transpose
    if (r < N && c < N) {
      hiT[(size_t)r * N + c] = th[tx][ty + 8 * q];
      loT[(size_t)r * N + c] = tl[tx][ty + 8 * q];
    }
  }
}

// transpose of an N x N double matrix
__global__ __launch_bounds__(256) void k_transpose64(int N, DSel<double> sel, double *AT)
{
  __shared__ double t[32][33];
  const double *A;
  double *unused;
  if (!resolve(sel, A, unused)) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + ty + 8 * q, c = c0 + tx;
    t[ty + 8 * q][tx] = (r < N && c < N) ? A[(size_t)r * N + c] : 0.0;
  }
  __syncthreads();
  for (int q = 0; q < 4; ++q) {
    const int r = c0 + ty + 8 * q, c = r0 + tx;
    if (r < N && c < N) AT[(size_t)r * N + c] = t[tx][ty + 8 * q];
  }
}

// ---- tile order of the GEMMs ---------------------------------------------------------
// Launch block b computes output tile (tr, tc) of an nt x nt grid of tiles (with
// SYM only those on and above the diagonal, tc >= tr).  The hardware deals the
// blocks to the chip's 8 XCDs in turn, so block b is first mapped to position
// t = (b mod 8) (nb / 8) + b / 8 of a single order, and each XCD runs a
// contiguous stretch of it; the order walks groups of kTileGroup tile rows
// column by column, so the blocks an XCD runs at once share a few row and
// column panels of the operands in its L2 instead of each reading its own.
constexpr int kXcds = 8, kTileGroup = 8;
__host__ __device__ inline int tile_count(int nt, bool sym) { return sym ? nt * (nt + 1) / 2 : nt * nt; }
__host__ __device__ inline void tile_of(int b, int nb, int nt, bool sym, int &tr, int &tc)
{
  const int per = nb / kXcds, full = per * kXcds;
  int t = b < full ? (b % kXcds) * per + b / kXcds : b;
  for (int r0 = 0; r0 < nt; r0 += kTileGroup) {
    const int rows = nt - r0 < kTileGroup ? nt - r0 : kTileGroup;
    const int tri = sym ? rows * (rows + 1) / 2 : 0;  // the group's tiles in its diagonal block (SYM)
    const int cnt = sym ? tri + rows * (nt - r0 - rows) : rows * nt;
    if (t >= cnt) {
      t -= cnt;
      continue;
    }
    if (!sym) {
      tc = t / rows;
      tr = r0 + t % rows;
    } else if (t < tri) {  // column r0 + m holds rows r0 .. r0 + m
      int m = 0;
      while ((m + 1) * (m + 2) / 2 <= t) ++m;
      tc = r0 + m;
      tr = r0 + (t - m * (m + 1) / 2);
    } else {
      t -= tri;
      tc = r0 + rows + t / rows;
      tr = r0 + t % rows;
    }
    return;
  }
  tr = tc = 0;  // (b < nb: not reached)
}

// ---- BF16x3 GEMM: C = hi.hi + hi.lo + lo.hi, 128 x 128 tile per block ----------------
// LDS holds 64 k-values per row (A tiles) and per column (B tiles, read from the
// transposed copies); the next 64-value slice is loaded into registers while
// the current one's products issue.  Wave (wm, wn) computes rows 64 wm .. +63 and columns
// 64 wn .. +63 as 2 x 2 MFMA 32 x 32 blocks.  v_mfma_f32_32x32x16_bf16 operand
// layout: lane l feeds A[l % 32][8 (l / 32) .. +7] and B[8 (l / 32) .. +7][l % 32]
// and holds C[8 g + 4 (l / 32) + t][l % 32] in accumulator 4 g + t.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kBM = 128, kBK = 64;
constexpr int kLdsK = kBK + 8;               // padded LDS row: 72 bf16 (144 bytes)
constexpr int kPieces = kBM * kBK / 8 / 256;  // 16-byte pieces of one tile per thread (4)

// One 16-byte piece (8 bf16 along k) of row `gr`, from k = gk; zeros past N.
// With VEC (N % 8 == 0) a raw buffer load over the N x N matrix, whose
// out-of-range offset reads zeros, so no branch separates the load from its use.
template <bool VEC>
__device__ __forceinline__ uint4 fetch_piece(int N, const uint16_t *__restrict__ src, __amdgpu_buffer_rsrc_t rs,
                                             int gr, int gk)
{
  if (VEC) {
    uint32_t off = gr < N && gk < N ? ((uint32_t)gr * (uint32_t)N + (uint32_t)gk) * 2u : 0xffffffffu;
    asm("" : "+v"(off));
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
    return make_uint4(v.x, v.y, v.z, v.w);
  }
  uint4 v = make_uint4(0, 0, 0, 0);
  if (gr < N) {
    uint16_t tmp[8];
    for (int e = 0; e < 8; ++e) tmp[e] = gk + e < N ? src[(size_t)gr * N + gk + e] : 0;
    memcpy(&v, tmp, 16);
  }
  return v;
}

// The four operand tiles (A hi, A lo from rows row0.., B hi, B lo from the
// transposed copies' rows col0..) of the k-slice k0 .. k0 + kBK - 1: thread t
// holds pieces t + 256 j, piece p = row p / 8, k-offset 8 (p % 8).
template <bool VEC>
__device__ __forceinline__ void fetch_tiles(int N, const uint16_t *const (&src)[4],
                                            const __amdgpu_buffer_rsrc_t (&rs)[4], int row0, int col0, int k0,
                                            uint4 (&pre)[4][kPieces])
{
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int j = 0; j < kPieces; ++j) {
      const int p = threadIdx.x + 256 * j;
      pre[t][j] = fetch_piece<VEC>(N, src[t], rs[t], (t < 2 ? row0 : col0) + (p >> 3), k0 + (p & 7) * 8);
    }
}

// SYM (X symmetric): X is its own transpose, so the B operands come from hi
// and lo themselves, and only the tiles on and above the diagonal are
// computed; k_mirror copies them below it (the split products hi.lo and lo.hi
// then give C a symmetric rounding as well).
template <bool VEC, bool SYM>
__global__ __launch_bounds__(256) void k_gemm_bf16x3(int N, const uint16_t *__restrict__ hi,
                                                     const uint16_t *__restrict__ lo,
                                                     const uint16_t *__restrict__ hiT,
                                                     const uint16_t *__restrict__ loT, DSel<float> sel)
{
  __shared__ __attribute__((aligned(16))) uint16_t T4[4][kBM][kLdsK];  // A hi, A lo, B hi, B lo
  int tr, tc;
  tile_of(blockIdx.x, gridDim.x, (N + kBM - 1) / kBM, SYM, tr, tc);
  const float *unused;
  float *C;
  if (!resolve(sel, unused, C)) return;
  if (SYM) {
    hiT = hi;
    loT = lo;
  }
  const int lane = lane_id(), w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int row0 = tr * kBM, col0 = tc * kBM;
  const uint16_t *const src[4] = {hi, lo, hiT, loT};
  const uint32_t bytes = (uint32_t)((size_t)N * N * 2 > 0xfffffff0u ? 0xfffffff0u : (size_t)N * N * 2);
  const __amdgpu_buffer_rsrc_t rs[4] = {
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(hi), (short)0, (int)bytes, 0x00020000),
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(lo), (short)0, (int)bytes, 0x00020000),
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(hiT), (short)0, (int)bytes, 0x00020000),
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(loT), (short)0, (int)bytes, 0x00020000)};
  f32x16 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 16; ++e) acc[a][b][e] = 0.f;
  uint4 pre[4][kPieces];
  auto stage = [&]() {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int j = 0; j < kPieces; ++j) {
        const int p = threadIdx.x + 256 * j;
        memcpy(&T4[t][p >> 3][(p & 7) * 8], &pre[t][j], 16);
      }
  };
  fetch_tiles<VEC>(N, src, rs, row0, col0, 0, pre);
  stage();
  __syncthreads();
  // the next slice's global loads are in flight while this slice's products issue
  for (int k0 = 0; k0 < N; k0 += kBK) {
    const bool more = k0 + kBK < N;
    if (more) fetch_tiles<VEC>(N, src, rs, row0, col0, k0 + kBK, pre);
    for (int ks = 0; ks < kBK; ks += 16) {
      const int kk = ks + 8 * (lane >> 5);
      bf16x8 ah[2], al[2], bh[2], bl[2];
      for (int a = 0; a < 2; ++a) {
        const int r = wm * 64 + a * 32 + (lane & 31);
        memcpy(&ah[a], &T4[0][r][kk], 16);
        memcpy(&al[a], &T4[1][r][kk], 16);
      }
      for (int b = 0; b < 2; ++b) {
        const int c = wn * 64 + b * 32 + (lane & 31);
        memcpy(&bh[b], &T4[2][c][kk], 16);
        memcpy(&bl[b], &T4[3][c][kk], 16);
      }
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
        }
    }
    __syncthreads();
    if (more) {
      stage();
      __syncthreads();
    }
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 16; ++e) {
        const int r = row0 + wm * 64 + a * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        const int c = col0 + wn * 64 + b * 32 + (lane & 31);
        if (r < N && c < N) C[(size_t)r * N + c] = acc[a][b][e];
      }
}

// ---- FP64 GEMM: C = A.A, 128 x 128 tile per block -----------------------------------
// v_mfma_f64_16x16x4_f64: lane l feeds A[l % 16][l / 16] and B[l / 16][l % 16]
// and holds C[l / 16 + 4 t][l % 16] in accumulator t.  Each output is updated by
// a chain of four fused multiply-adds in ascending k (checked on gfx950 against
// exactly rounded fma on random operands), so with k0 ascending the whole
// product is the same fma chain as the textbook loop, bit for bit.  Wave
// (wm, wn) owns rows 64 wm .. +63 and columns 64 wn .. +63 (4 x 4 MFMA blocks).
constexpr int kDM = 128, kDK = 16;
constexpr int kDPieces = kDM * kDK / 2 / 256;  // 16-byte pieces (two doubles) of one tile per thread (4)

// Piece p of the k-slice k0 .. k0 + kDK - 1 of rows row0..: row p / 8, k-offset
// 2 (p % 8).  With VEC (N even) one raw buffer load whose out-of-range offset
// reads zeros; else element by element.
template <bool VEC>
__device__ __forceinline__ void fetch_pair(int N, const double *__restrict__ src, __amdgpu_buffer_rsrc_t rs,
                                           int gr, int gk, double &v0, double &v1)
{
  if (VEC) {
    uint32_t off = gr < N && gk < N ? ((uint32_t)gr * (uint32_t)N + (uint32_t)gk) * 8u : 0xffffffffu;
    asm("" : "+v"(off));
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
    v0 = __builtin_bit_cast(double, (unsigned long long)v.y << 32 | v.x);
    v1 = __builtin_bit_cast(double, (unsigned long long)v.w << 32 | v.z);
    return;
  }
  v0 = gr < N && gk < N ? src[(size_t)gr * N + gk] : 0.0;
  v1 = gr < N && gk + 1 < N ? src[(size_t)gr * N + gk + 1] : 0.0;
}

// SYM (X bitwise symmetric): X is its own transpose, and C = X.X is bitwise
// symmetric (C_ji sums the products of C_ij in the same k order), so only the
// tiles on and above the diagonal are computed; k_mirror copies them below it,
// with the same bits as the whole product.
template <bool VEC, bool SYM>
__global__ __launch_bounds__(256) void k_gemm_f64(int N, const double *__restrict__ AT, DSel<double> sel)
{
  __shared__ double As[kDM][kDK + 1], Bs[kDM][kDK + 1];
  int tr, tc;
  tile_of(blockIdx.x, gridDim.x, (N + kDM - 1) / kDM, SYM, tr, tc);
  const double *A;
  double *C;
  if (!resolve(sel, A, C)) return;
  if (SYM) AT = A;
  const int lane = lane_id(), w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int row0 = tr * kDM, col0 = tc * kDM;
  const size_t nbytes = (size_t)N * N * 8;
  const uint32_t bytes = (uint32_t)(nbytes > 0xfffffff0u ? 0xfffffff0u : nbytes);
  const __amdgpu_buffer_rsrc_t ra =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(A), (short)0, (int)bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rb =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(AT), (short)0, (int)bytes, 0x00020000);
  f64x4 acc[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int e = 0; e < 4; ++e) acc[a][b][e] = 0.0;
  double pa[kDPieces][2], pb[kDPieces][2];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int j = 0; j < kDPieces; ++j) {
      const int p = threadIdx.x + 256 * j;
      fetch_pair<VEC>(N, A, ra, row0 + (p >> 3), k0 + 2 * (p & 7), pa[j][0], pa[j][1]);
      fetch_pair<VEC>(N, AT, rb, col0 + (p >> 3), k0 + 2 * (p & 7), pb[j][0], pb[j][1]);
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int j = 0; j < kDPieces; ++j) {
      const int p = threadIdx.x + 256 * j;
      const int r = p >> 3, k = 2 * (p & 7);
      As[r][k] = pa[j][0];
      As[r][k + 1] = pa[j][1];
      Bs[r][k] = pb[j][0];
      Bs[r][k + 1] = pb[j][1];
    }
  };
  fetch(0);
  stage();
  __syncthreads();
  // the next slice's loads are in flight while this slice's products issue
  for (int k0 = 0; k0 < N; k0 += kDK) {
    const bool more = k0 + kDK < N;
    if (more) fetch(k0 + kDK);
    for (int ks = 0; ks < kDK; ks += 4) {
      const int kk = ks + (lane >> 4);
      double av[4], bv[4];
      for (int a = 0; a < 4; ++a) av[a] = As[wm * 64 + a * 16 + (lane & 15)][kk];
      for (int b = 0; b < 4; ++b) bv[b] = Bs[wn * 64 + b * 16 + (lane & 15)][kk];
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
    if (more) {
      stage();
      __syncthreads();
    }
  }
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int e = 0; e < 4; ++e) {
        const int r = row0 + wm * 64 + a * 16 + (lane >> 4) + 4 * e;
        const int c = col0 + wn * 64 + b * 16 + (lane & 15);
        if (r < N && c < N) C[(size_t)r * N + c] = acc[a][b][e];
      }
}

// The part of C below the GEMM's diagonal tiles (row tile above column tile,
// in tiles of TILE) from its transpose above them, 32 x 32 blocks through LDS.
template <typename T, int TILE>
__global__ __launch_bounds__(256) void k_mirror(int N, DSel<T> sel)
{
  __shared__ T t[32][33];
  if ((int)(blockIdx.y * 32) / TILE <= (int)(blockIdx.x * 32) / TILE) return;  // computed by the GEMM
  const T *unused;
  T *C;
  if (!resolve(sel, unused, C)) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;  // the block to fill
  for (int q = 0; q < 4; ++q) {
    const int r = c0 + ty + 8 * q, c = r0 + tx;  // its transpose
    t[ty + 8 * q][tx] = (r < N && c < N) ? C[(size_t)r * N + c] : T(0);
  }
  __syncthreads();
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + ty + 8 * q, c = c0 + tx;
    if (r < N && c < N) C[(size_t)r * N + c] = t[tx][ty + 8 * q];
  }
}

// ---- per-row step outputs: U = 2X - Y, diagonals, norm row term ---------------------
// One wave per row.  The norm's row term is the pairwise tree over the N column
// positions, evaluated as the perfect tree over 64-column blocks (lane tree),
// then over groups of 64 blocks, then over the (at most 64) groups; positions
// past N contribute +0, the exact identity for these non-negative terms.
template <typename T>
__global__ __launch_bounds__(256) void k_dense_rows(int N, T *const *bufs, const SP2State *st, StepScratch s)
{
  __shared__ double gs[4][kWave];
  if (st->stop) return;
  const int cur = st->cur;
  const T *X = bufs[cur];
  const T *Y = bufs[cur == 2 ? 0 : cur + 1];
  T *U = bufs[cur == 0 ? 2 : cur - 1];
  const int w = threadIdx.x >> 6, lane = lane_id();
  const int i = blockIdx.x * 4 + w;
  if (i >= N) return;  // whole wave: i is wave-uniform
  const int nblk = (N + kWave - 1) / kWave;
  const int ngrp = (nblk + kWave - 1) / kWave;
  for (int g = 0; g < ngrp; ++g) {
    double mine = 0.0;
    for (int b = g * kWave; b < min(nblk, (g + 1) * kWave); ++b) {
      const int j = b * kWave + lane;
      double q = 0.0;
      if (j < N) {
        const T x = X[(size_t)i * N + j], y = Y[(size_t)i * N + j];
        U[(size_t)i * N + j] = T(2) * x - y;
        const double d = (double)y - (double)x;
        q = d * d;
        if (j == i) {
          s.d1[i] = (double)x;
          s.d2[i] = (double)y;
        }
      }
      const double t = __shfl(wave_tree(q), 0, kWave);
      if (lane == b - g * kWave) mine = t;
    }
    const double gsum = wave_tree(mine);
    if (lane == 0) gs[w][g] = gsum;
  }
  const double v = lane < ngrp ? gs[w][lane] : 0.0;
  const double total = wave_tree(v);
  if (lane == 0) {
    s.e[i] = total;
    s.wy[i] = 0;
    s.wu[i] = 0;
  }
}

// Gershgorin bounds per row: H_ii -/+ the sum over j != i of |H_ij|, ascending j
__global__ __launch_bounds__(256) void k_dense_gersh(int N, const double *__restrict__ H, double *lo_out,
                                                     double *hi_out)
{
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  double r = 0.0;
  for (int j = 0; j < N; ++j)
    if (j != i) r = r + fabs(H[(size_t)i * N + j]);
  const double h = H[(size_t)i * N + i];
  lo_out[i] = h - r;
  hi_out[i] = h + r;
}

// X0 = (emax I - H) / (emax - emin), with inv = 1 / (emax - emin)
template <typename T>
__global__ __launch_bounds__(256) void k_dense_x0(int N, const double *__restrict__ H, T *X, double emax, double inv)
{
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (size_t)N * N) return;
  const int i = (int)(q / N), j = (int)(q % N);
  const double h = H[q];
  const double x = (j == i) ? (emax - h) * inv : (-h) * inv;
  X[q] = (T)x;
}

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_dense_copy(size_t n, const TS *__restrict__ a, TD *b)
{
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q < n) b[q] = (TD)a[q];
}

struct DMem {
  void *p = nullptr;
  ~DMem() { if (p) (void)hipFree(p); }
  hipError_t alloc(size_t n) { return hipMalloc(&p, n ? n : 1); }
};

#define DTRY(expr)                                          \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return device_error(e_, #expr);   \
  } while (0)

// sym: X is bitwise symmetric (no transposed copies; the upper triangle of
// tiles, mirrored)
hipError_t product_f32(int N, DSel<float> sel, uint16_t *hi, uint16_t *lo, uint16_t *hiT, uint16_t *loT,
                       hipStream_t s, bool sym = false)
{
  const dim3 tb((N + 31) / 32, (N + 31) / 32);
  hipLaunchKernelGGL(k_split, tb, dim3(256), 0, s, N, sel, hi, lo, sym ? nullptr : hiT, sym ? nullptr : loT);
  const dim3 gb(tile_count((N + kBM - 1) / kBM, sym));
  if (N % 8 == 0) {
    if (sym) hipLaunchKernelGGL((k_gemm_bf16x3<true, true>), gb, dim3(256), 0, s, N, hi, lo, hiT, loT, sel);
    else hipLaunchKernelGGL((k_gemm_bf16x3<true, false>), gb, dim3(256), 0, s, N, hi, lo, hiT, loT, sel);
  } else {
    if (sym) hipLaunchKernelGGL((k_gemm_bf16x3<false, true>), gb, dim3(256), 0, s, N, hi, lo, hiT, loT, sel);
    else hipLaunchKernelGGL((k_gemm_bf16x3<false, false>), gb, dim3(256), 0, s, N, hi, lo, hiT, loT, sel);
  }
  if (sym) hipLaunchKernelGGL((k_mirror<float, kBM>), tb, dim3(256), 0, s, N, sel);
  return hipGetLastError();
}

hipError_t product_f64(int N, DSel<double> sel, double *XT, hipStream_t s, bool sym = false)
{
  const dim3 tb((N + 31) / 32, (N + 31) / 32);
  if (!sym) hipLaunchKernelGGL(k_transpose64, tb, dim3(256), 0, s, N, sel, XT);
  const dim3 gb(tile_count((N + kDM - 1) / kDM, sym));
  if (N % 2 == 0) {
    if (sym) hipLaunchKernelGGL((k_gemm_f64<true, true>), gb, dim3(256), 0, s, N, XT, sel);
    else hipLaunchKernelGGL((k_gemm_f64<true, false>), gb, dim3(256), 0, s, N, XT, sel);
  } else {
    if (sym) hipLaunchKernelGGL((k_gemm_f64<false, true>), gb, dim3(256), 0, s, N, XT, sel);
    else hipLaunchKernelGGL((k_gemm_f64<false, false>), gb, dim3(256), 0, s, N, XT, sel);
  }
  if (sym) hipLaunchKernelGGL((k_mirror<double, kDM>), tb, dim3(256), 0, s, N, sel);
  return hipGetLastError();
}

// flag |= 1 if some A[r][c] and A[c][r] differ in their bits (32 x 32 tiles)
__global__ __launch_bounds__(256) void k_dense_asym(int N, const double *__restrict__ A, int32_t *flag)
{
  __shared__ double t[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  if (blockIdx.y > blockIdx.x) return;  // each pair of tiles once
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + ty + 8 * q, c = c0 + tx;
    t[ty + 8 * q][tx] = (r < N && c < N) ? A[(size_t)r * N + c] : 0.0;
  }
  __syncthreads();
  bool bad = false;
  for (int q = 0; q < 4; ++q) {
    const int r = c0 + ty + 8 * q, c = r0 + tx;  // A[r][c] against A[c][r] of the tile above
    if (r < N && c < N)
      bad |= __double_as_longlong(A[(size_t)r * N + c]) != __double_as_longlong(t[tx][ty + 8 * q]);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

}  // namespace
}  // namespace ellsp2

using namespace ellsp2;

extern "C" int dense_x2(const void *d_A, void *d_C, int32_t N, int32_t mode, void *hip_stream)
{
  if (!d_A || !d_C || N <= 0 || N > kMaxDenseN || d_A == d_C) return ELL_EINVAL;
  if (mode != DENSE_F64 && mode != DENSE_BF16X3) return ELL_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const size_t nn = (size_t)N * N;
  if (mode == DENSE_BF16X3) {
    DMem hi, lo, hiT, loT;
    DTRY(hi.alloc(nn * 2));
    DTRY(lo.alloc(nn * 2));
    DTRY(hiT.alloc(nn * 2));
    DTRY(loT.alloc(nn * 2));
    DSel<float> sel{(const float *)d_A, (float *)d_C, nullptr, nullptr};
    DTRY(product_f32(N, sel, (uint16_t *)hi.p, (uint16_t *)lo.p, (uint16_t *)hiT.p, (uint16_t *)loT.p, s));
    DTRY(hipStreamSynchronize(s));
  } else {
    DMem at;
    DTRY(at.alloc(nn * 8));
    DSel<double> sel{(const double *)d_A, (double *)d_C, nullptr, nullptr};
    DTRY(product_f64(N, sel, (double *)at.p, s));
    DTRY(hipStreamSynchronize(s));
  }
  return ELL_OK;
}

extern "C" int dense_sp2_solve(const double *d_H, int32_t N, double *d_D, int32_t mode, const sp2_params_t *p,
                               sp2_report_t *r, void *hip_stream)
{
  if (!d_H || !d_D || N <= 0 || N > kMaxDenseN || !p || (const void *)d_H == (const void *)d_D) return ELL_EINVAL;
  if (mode != DENSE_F64 && mode != DENSE_BF16X3) return ELL_EINVAL;
  if (!(p->idem_target >= 0.0) || p->max_iter < 1 || p->fp64_tail_steps < 0 || !std::isfinite(p->n_occ))
    return ELL_EINVAL;
  if (r) {
    r->status = 0;
    r->iterations = r->fp32_iterations = r->final_M = 0;
    r->eta = r->trace_x = r->emin = r->emax = r->seconds = r->x2_seconds = 0.0;
    r->x2_bytes = 0;
    r->x2_launches = 0;
    r->batch_k = r->batch_kernel = 0;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const size_t nn = (size_t)N * N;
  const bool lowp = mode == DENSE_BF16X3;

  // Gershgorin bounds: per-row bounds on the device, min / max (exact) on the host
  DMem glo, ghi;
  DTRY(glo.alloc(sizeof(double) * N));
  DTRY(ghi.alloc(sizeof(double) * N));
  hipLaunchKernelGGL(k_dense_gersh, dim3((N + 255) / 256), dim3(256), 0, s, N, d_H, (double *)glo.p,
                     (double *)ghi.p);
  DTRY(hipGetLastError());
  // a bitwise symmetric H keeps every iterate bitwise symmetric (X0 is; X^2
  // sums the same products for (i, j) and (j, i); 2X - X^2 is entrywise): the
  // products then take the upper triangle of tiles only
  DMem asym;
  DTRY(asym.alloc(sizeof(int32_t)));
  DTRY(hipMemsetAsync(asym.p, 0, sizeof(int32_t), s));
  hipLaunchKernelGGL(k_dense_asym, dim3((N + 31) / 32, (N + 31) / 32), dim3(256), 0, s, N, d_H,
                     (int32_t *)asym.p);
  DTRY(hipGetLastError());
  std::vector<double> hlo(N), hhi(N);
  int32_t hasym = 0;
  DTRY(hipMemcpyAsync(hlo.data(), glo.p, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  DTRY(hipMemcpyAsync(hhi.data(), ghi.p, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  DTRY(hipMemcpyAsync(&hasym, asym.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  DTRY(hipStreamSynchronize(s));
  const bool sym = hasym == 0;
  double emin = INFINITY, emax = -INFINITY;
  for (int i = 0; i < N; ++i) {
    if (!std::isfinite(hlo[i]) || !std::isfinite(hhi[i])) return ELL_ENONFINITE;
    emin = std::min(emin, hlo[i]);
    emax = std::max(emax, hhi[i]);
  }
  if (r) {
    r->emin = emin;
    r->emax = emax;
  }
  if (!(emax > emin)) return ELL_EDEGENERATE;
  if (!(p->n_occ > 0.0 && p->n_occ < (double)N)) return ELL_EDEGENERATE;
  const double inv = 1.0 / (emax - emin);

  // working matrices: three of each precision in use, rotated by the device state
  DMem b32[3], b64[3], hi, lo, hiT, loT, xt, ptrs32, ptrs64;
  if (lowp) {
    for (auto &b : b32) DTRY(b.alloc(nn * 4));
    DTRY(hi.alloc(nn * 2));
    DTRY(lo.alloc(nn * 2));
    if (!sym) {  // (transposed copies: a symmetric X is its own transpose)
      DTRY(hiT.alloc(nn * 2));
      DTRY(loT.alloc(nn * 2));
    }
  }
  for (auto &b : b64) DTRY(b.alloc(nn * 8));
  if (!sym) DTRY(xt.alloc(nn * 8));
  float *p32[3] = {(float *)b32[0].p, (float *)b32[1].p, (float *)b32[2].p};
  double *p64[3] = {(double *)b64[0].p, (double *)b64[1].p, (double *)b64[2].p};
  DTRY(ptrs32.alloc(sizeof(p32)));
  DTRY(ptrs64.alloc(sizeof(p64)));
  DTRY(hipMemcpyAsync(ptrs32.p, p32, sizeof(p32), hipMemcpyHostToDevice, s));
  DTRY(hipMemcpyAsync(ptrs64.p, p64, sizeof(p64), hipMemcpyHostToDevice, s));

  // step scratch and device state
  const int nb = (N + kRedBlock - 1) / kRedBlock;
  const size_t mi = (size_t)p->max_iter;
  DMem d1, d2, e, wy, wu, part, partw, partn, out, outw, outn, state, h_trx, h_trx2, h_eta2, h_up, h_prec, h_maxw,
      h_nx, h_ny;
  DTRY(d1.alloc(8 * (size_t)N));
  DTRY(d2.alloc(8 * (size_t)N));
  DTRY(e.alloc(8 * (size_t)N));
  DTRY(wy.alloc(4 * (size_t)N));
  DTRY(wu.alloc(4 * (size_t)N));
  DTRY(part.alloc(8 * 3 * (size_t)nb));
  DTRY(partw.alloc(4 * 4 * (size_t)nb));
  DTRY(partn.alloc(8 * 2 * (size_t)nb));
  DTRY(out.alloc(8 * 3));
  DTRY(outw.alloc(4 * 4));
  DTRY(outn.alloc(8 * 2));
  DTRY(state.alloc(sizeof(SP2State)));
  DTRY(h_trx.alloc(8 * mi));
  DTRY(h_trx2.alloc(8 * mi));
  DTRY(h_eta2.alloc(8 * mi));
  DTRY(h_up.alloc(mi));
  DTRY(h_prec.alloc(mi));
  DTRY(h_maxw.alloc(4 * mi));
  DTRY(h_nx.alloc(8 * mi));
  DTRY(h_ny.alloc(8 * mi));
  StepScratch sc{};
  sc.d1 = (double *)d1.p;
  sc.d2 = (double *)d2.p;
  sc.e = (double *)e.p;
  sc.wy = (int32_t *)wy.p;
  sc.wu = (int32_t *)wu.p;
  sc.part = (double *)part.p;
  sc.partw = (int32_t *)partw.p;
  sc.partn = (int64_t *)partn.p;
  sc.out = (double *)out.p;
  sc.outw = (int32_t *)outw.p;
  sc.outn = (int64_t *)outn.p;
  sc.nb = nb;
  SP2Hist hist{(double *)h_trx.p, (double *)h_trx2.p, (double *)h_eta2.p, (int8_t *)h_up.p,
               (int8_t *)h_prec.p, (int32_t *)h_maxw.p, (int64_t *)h_nx.p, (int64_t *)h_ny.p};
  SP2Cfg cfg{};
  cfg.n_occ = p->n_occ;
  cfg.target2 = p->idem_target * p->idem_target;
  cfg.switch2 = p->switch_eta * p->switch_eta;
  cfg.max_iter = p->max_iter;
  cfg.tail = p->fp64_tail_steps;
  cfg.stall = p->stall_stop ? 1 : 0;
  cfg.mixed = lowp ? 1 : 0;
  cfg.span = 0;

  std::vector<hipEvent_t> ev(2 + (p->profile ? 2 * (size_t)std::max(1, p->poll_every) : 0), nullptr);
  struct EvList {
    std::vector<hipEvent_t> &v;
    ~EvList()
    {
      for (auto x : v)
        if (x) (void)hipEventDestroy(x);
    }
  } evl{ev};
  for (auto &x : ev) DTRY(hipEventCreate(&x));
  hipEvent_t t0 = ev[0], t1 = ev[1];
  DTRY(hipEventRecord(t0, s));
  const unsigned eb = (unsigned)((nn + 255) / 256);
  if (lowp)
    hipLaunchKernelGGL((k_dense_x0<float>), dim3(eb), dim3(256), 0, s, N, d_H, p32[0], emax, inv);
  else
    hipLaunchKernelGGL((k_dense_x0<double>), dim3(eb), dim3(256), 0, s, N, d_H, p64[0], emax, inv);
  DTRY(hipGetLastError());
  SP2State hs{};
  hs.status = ST_RUNNING;
  hs.phase32 = lowp ? 1 : 0;
  hs.cap = INT_MAX;
  hs.sw = INT_MAX;
  hs.nnz_cur = (int64_t)nn;
  SP2State *dst = (SP2State *)state.p;
  DTRY(hipMemcpyAsync(dst, &hs, sizeof(hs), hipMemcpyHostToDevice, s));
  const int poll = p->poll_every > 0 ? p->poll_every : 1;
  const dim3 rowgrid((N + 3) / 4);
  DSel<float> sel32{nullptr, nullptr, (float *const *)ptrs32.p, dst};
  DSel<double> sel64{nullptr, nullptr, (double *const *)ptrs64.p, dst};
  double x2_sec = 0.0;
  int32_t x2_n = 0;
  int64_t x2_bytes = 0;
  int status = ST_RUNNING;
  for (int64_t batch = 0;; ++batch) {
    if (batch > (int64_t)p->max_iter + 8) {
      set_device_error("dense_sp2_solve: the device state did not reach a stop");
      return ELL_EDEVICE;
    }
    const int iter0 = hs.iter;
    for (int q = 0; q < poll; ++q) {
      if (p->profile) DTRY(hipEventRecord(ev[2 + 2 * q], s));
      if (hs.phase32)
        DTRY(product_f32(N, sel32, (uint16_t *)hi.p, (uint16_t *)lo.p, (uint16_t *)hiT.p, (uint16_t *)loT.p, s,
                         sym));
      else
        DTRY(product_f64(N, sel64, (double *)xt.p, s, sym));
      if (p->profile) DTRY(hipEventRecord(ev[3 + 2 * q], s));
      if (hs.phase32)
        hipLaunchKernelGGL((k_dense_rows<float>), rowgrid, dim3(256), 0, s, N, (float *const *)ptrs32.p, dst, sc);
      else
        hipLaunchKernelGGL((k_dense_rows<double>), rowgrid, dim3(256), 0, s, N, (double *const *)ptrs64.p, dst,
                           sc);
      DTRY(hipGetLastError());
      DTRY(launch_reduce(N, dst, sc, s));
      DTRY(launch_decide(dst, cfg, hist, sc, s));
    }
    const int phase32 = hs.phase32;
    DTRY(hipMemcpyAsync(&hs, dst, sizeof(hs), hipMemcpyDeviceToHost, s));
    DTRY(hipStreamSynchronize(s));
    if (p->profile) {  // products that ran: one per decision taken in this batch
      const int ran = std::min(poll, hs.iter - iter0);
      for (int q = 0; q < ran; ++q) {
        float ms = 0.f;
        DTRY(hipEventElapsedTime(&ms, ev[2 + 2 * q], ev[3 + 2 * q]));
        x2_sec += ms * 1e-3;
        if (r && r->hist_x2_seconds && x2_n < p->max_iter) r->hist_x2_seconds[x2_n] = ms * 1e-3;
        if (r && r->hist_x2_bytes && x2_n < p->max_iter) r->hist_x2_bytes[x2_n] = (int64_t)nn * (phase32 ? 8 : 16);
        ++x2_n;
        // algorithmic traffic of one product: X read once, X^2 written once
        x2_bytes += (int64_t)nn * (phase32 ? 8 : 16);
      }
    }
    if (!hs.stop) continue;
    if (hs.status == ST_SWITCH) {
      // widen the current FP32 X into FP64 buffer 0 and go on in FP64
      hipLaunchKernelGGL((k_dense_copy<float, double>), dim3(eb), dim3(256), 0, s, nn, p32[hs.cur], p64[0]);
      DTRY(hipGetLastError());
      hs.cur = 0;
      hs.phase32 = 0;
      hs.stop = 0;
      hs.status = ST_RUNNING;
      DTRY(hipMemcpyAsync(dst, &hs, sizeof(hs), hipMemcpyHostToDevice, s));
      continue;
    }
    status = hs.status;
    break;
  }
  DTRY(hipEventRecord(t1, s));
  // the returned X, in double
  if (hs.phase32)
    hipLaunchKernelGGL((k_dense_copy<float, double>), dim3(eb), dim3(256), 0, s, nn, p32[hs.cur], d_D);
  else
    hipLaunchKernelGGL((k_dense_copy<double, double>), dim3(eb), dim3(256), 0, s, nn, p64[hs.cur], d_D);
  DTRY(hipGetLastError());
  DTRY(hipStreamSynchronize(s));
  if (r) {
    const int n = hs.iter;
    r->status = status;
    r->iterations = n;
    r->final_M = N;
    r->eta = std::sqrt(hs.eta2);
    r->trace_x = hs.trx;
    float ms = 0.f;
    DTRY(hipEventElapsedTime(&ms, t0, t1));
    r->seconds = ms * 1e-3;
    std::vector<double> va(n), vb(n), vc(n);
    std::vector<int8_t> vu(n), vp(n);
    if (n > 0) {
      DTRY(hipMemcpy(va.data(), h_trx.p, 8 * (size_t)n, hipMemcpyDeviceToHost));
      DTRY(hipMemcpy(vb.data(), h_trx2.p, 8 * (size_t)n, hipMemcpyDeviceToHost));
      DTRY(hipMemcpy(vc.data(), h_eta2.p, 8 * (size_t)n, hipMemcpyDeviceToHost));
      DTRY(hipMemcpy(vu.data(), h_up.p, (size_t)n, hipMemcpyDeviceToHost));
      DTRY(hipMemcpy(vp.data(), h_prec.p, (size_t)n, hipMemcpyDeviceToHost));
    }
    int f32 = 0;
    for (int q = 0; q < n; ++q) {
      f32 += vp[q] ? 1 : 0;
      if (r->hist_trx) r->hist_trx[q] = va[q];
      if (r->hist_trx2) r->hist_trx2[q] = vb[q];
      if (r->hist_eta2) r->hist_eta2[q] = vc[q];
      if (r->hist_up) r->hist_up[q] = vu[q];
      if (r->hist_prec) r->hist_prec[q] = vp[q];
      if (r->hist_maxw) r->hist_maxw[q] = N;
    }
    r->fp32_iterations = f32;
    r->x2_seconds = x2_sec;
    r->x2_launches = x2_n;
    r->x2_bytes = x2_bytes;
  }
  return status;
}
