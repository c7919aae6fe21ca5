// Wavefront helpers shared by the span-form X^2 kernels (ell_band.hip,
// ell_band16.hip).  Device-only; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ellsp2 {
namespace band {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }
// a value every lane holds, moved to a scalar register
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int lanes_below(uint64_t m)
{
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ void wave_sync()
{
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ int wmin(int v)
{
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ int wmax(int v)
{
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
  return v;
}
// pairwise tree over the 64 lanes (lane l = leaf l); the total lands in lane 0
__device__ __forceinline__ double wave_tree(double v)
{
  for (int s = 1; s < kWave; s <<= 1) v = v + __shfl_down(v, s, kWave);
  return v;
}

// Consecutive workgroups go to the 8 XCDs in turn; remap so that each XCD
// works on one contiguous range of row groups (its own L2 then holds the rows
// k those groups share).
__device__ __forceinline__ int xcd_block(int b, int nblocks)
{
  constexpr int kXcd = 8;
  const int per = nblocks / kXcd;
  const int full = per * kXcd;
  if (b >= full) return b;
  return (b % kXcd) * per + b / kXcd;
}

// Raw buffer resources (stride 0): a lane whose byte offset is at or past the
// range reads 0, and its store is dropped.
constexpr int kRawBufferFlags = 0x00020000;  // 32-bit raw buffer, gfx9 family

}  // namespace band
}  // namespace ellsp2
