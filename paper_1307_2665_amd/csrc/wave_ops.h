// Wave-level helpers shared by the register-resident elimination kernels
// (merge panels and leaf panels): pivot search keys, a wave-wide unsigned
// max, a lane broadcast of a double and wave-local LDS ordering.  Device code
// only; included by .hip files.
#pragma once

#include <hip/hip_runtime.h>

namespace hps {

// Search key of a pivot candidate: |v| rounded to float (NaN as +inf) with
// the low 12 bits replaced by 4095 - slot, so one unsigned max finds both
// the largest magnitude (to 2^-11 relative) and where it lives.  0 = none.
__device__ inline unsigned pivot_key(double v, int slot) {
  const unsigned u = (v != v) ? 0x7F800000u : __float_as_uint((float)fabs(v));
  return (u & ~4095u) | (unsigned)(4095 - slot);
}

// Wave-wide unsigned max: DPP within each row of 16 lanes (quad swaps, then
// row rotations by 4 and 8), then the four row results through readlane.
__device__ inline unsigned wave_max_u32(unsigned k) {
  k = max(k, (unsigned)__builtin_amdgcn_mov_dpp((int)k, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  k = max(k, (unsigned)__builtin_amdgcn_mov_dpp((int)k, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  k = max(k, (unsigned)__builtin_amdgcn_mov_dpp((int)k, 0x124, 0xF, 0xF, false));  // row_ror:4
  k = max(k, (unsigned)__builtin_amdgcn_mov_dpp((int)k, 0x128, 0xF, 0xF, false));  // row_ror:8
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)k, 0);
  const unsigned b = (unsigned)__builtin_amdgcn_readlane((int)k, 16);
  const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)k, 32);
  const unsigned d = (unsigned)__builtin_amdgcn_readlane((int)k, 48);
  return max(max(a, b), max(c, d));
}

// Orders a wave's LDS accesses: what one lane wrote before is visible to
// every lane of the wave after it.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Broadcast of lane `src` (wave-uniform) of a double to the whole wave.
__device__ inline double bcast_lane(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// A double that is the same in every lane, moved to scalar registers.
__device__ inline double uniform(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(unsigned)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// 1/x for a finite nonzero x: the hardware reciprocal refined by two Newton
// steps (r <- r + r (1 - x r)), within an ulp of the quotient; magnitudes
// outside [1e-290, 1e290] take the division.
__device__ inline double recip(double x) {
  const double a = fabs(x);
  if (a > 1e-290 && a < 1e290) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
  }
  return 1.0 / x;
}

}  // namespace hps
