// Helpers shared by the matrix-core span kernels (ell_band16.hip,
// ell_sym16.hip): raw buffer loads and stores with range-checked offsets, the
// FP64 / FP32 16x16x4 matrix instructions, row bookkeeping of the span output
// and the perfect pairwise trees of the reductions.  Device-only; not part of
// the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>

#include "band_common.h"

namespace ellsp2 {
namespace span16 {

using band::kWave;

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr uint32_t kOob = 0x80000000u;  // byte offset past every buffer: loads give 0, stores are dropped

// Loads and stores through raw buffers.  The whole offset stays in the VGPR
// operand (no folding into the immediate or scalar offset fields, which the
// range check treats differently).
__device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, uint32_t off, double)
{
  asm("" : "+v"(off));
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t off, float)
{
  asm("" : "+v"(off));
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t off, double v)
{
  asm("" : "+v"(off));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t off, float v)
{
  asm("" : "+v"(off));
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ double absv(double a) { return __builtin_fabs(a); }
__device__ __forceinline__ float absv(float a) { return __builtin_fabsf(a); }

// byte offset of element e when `ok`, else past the buffer
template <typename T>
__device__ __forceinline__ uint32_t at(bool ok, int e)
{
  return ok ? (uint32_t)e * (uint32_t)sizeof(T) : kOob;
}

// The matrix instruction of each precision, and the output row its
// accumulator t holds in lane (r, q) = (l % 16, l / 16).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef f64x4 acc;
  static __device__ __forceinline__ acc mma(double a, double b, acc c)
  {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int t) { return q + 4 * t; }
};
template <> struct Mfma<float> {
  typedef f32x4 acc;
  static __device__ __forceinline__ acc mma(float a, float b, acc c)
  {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int t) { return 4 * q + t; }
};

// the 16 bits of a wave mask that belong to this lane's 16-lane row
__device__ __forceinline__ uint32_t seg16(uint64_t m, int q) { return (uint32_t)(m >> (16 * q)) & 0xffffu; }

// A lane's partner value through DPP: quad_perm [1,0,3,2] (0xb1) and
// [2,3,0,1] (0x4e) pair lanes 4m + (0,1), (2,3) and then the two pairs of a
// quad; with a + b = b + a exactly, both lanes of a pair get the same sum.
template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, false);
}

// Running output state of one row: first and last kept column, kept count.
// Blocks come in ascending column order.  A row's span output holds exactly
// its interval [first, last]: a block writes its columns from `first` up to
// its own last kept column, and when a block keeps something after blocks
// that kept nothing, the columns between get their zeros then.
struct RowRun {
  int first = INT_MAX, last = -1, count = 0;
  // lo, hi: kept columns p0 .. p0 + 31 and p0 + 32 .. p0 + 63 of this block.
  // Returns the last column the block writes (p0 - 1: none) and, in
  // gap_lo .. p0 - 1, the earlier columns that still need zeros.
  __device__ int add(uint32_t lo, uint32_t hi, int p0, int &gap_lo)
  {
    const bool any = (lo | hi) != 0;
    gap_lo = any && last >= 0 ? last + 1 : p0;
    count += __popc(lo) + __popc(hi);
    const int f = lo ? p0 + __ffs(lo) - 1 : hi ? p0 + 31 + __ffs(hi) : INT_MAX;
    first = min(first, f);
    const int l = hi ? p0 + 63 - __clz(hi) : p0 + 31 - __clz(lo);  // p0 - 1 when none
    last = any ? l : last;
    return l;
  }
  __device__ int length() const { return last >= 0 ? last - first + 1 : 0; }
};


// Perfect pairwise tree over p[a .. a + L); positions at or past n count as
// -0.0, the exact additive identity (x + -0.0 == x for every x).
template <int L>
__device__ __forceinline__ double leaf_tree(const double *p, int a, int n)
{
  if constexpr (L == 1) {
    return a < n ? p[a] : -0.0;
  } else {
    const double lo = leaf_tree<L / 2>(p, a, n);
    return lo + leaf_tree<L / 2>(p, a + L / 2, n);
  }
}

// The leaves of thread t for the three sums p[c nq .. c nq + nq), c = 0..2,
// as subtrees of one perfect tree per sum: thread t holds [a, a + L), a = t L,
// L the smallest power of two with 256 L >= nq (nq <= 16384); the trees over
// the threads follow.
template <int L>
__device__ __forceinline__ double leaf_tree_lean(const double *p, int a, int n)
{
  if constexpr (L <= 8) {
    return leaf_tree<L>(p, a, n);
  } else {  // halves one after the other: at most 8 leaves live at a time
    const double lo = leaf_tree_lean<L / 2>(p, a, n);
    asm volatile("" ::: "memory");
    return lo + leaf_tree_lean<L / 2>(p, a + L / 2, n);
  }
}

template <int L>
__device__ __forceinline__ void leaf_tree3(const double *p, int nq, int a, double (&v)[3])
{
  if constexpr (L <= 8) {
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = leaf_tree<L>(p + (size_t)c * nq, a, nq);
  } else {
#pragma unroll 1
    for (int c = 0; c < 3; ++c) v[c] = leaf_tree_lean<L>(p + (size_t)c * nq, a, nq);
  }
}

__device__ __forceinline__ long long wsum(long long v)
{
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

}  // namespace span16
}  // namespace ellsp2
