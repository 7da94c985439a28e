// Wavefront reductions built from DPP lane permutations (gfx9 encodings)
// and readlane: no LDS traffic, a few cycles per step.  Every lane of the
// wavefront must be active when they are called.
#pragma once

#include <hip/hip_runtime.h>

namespace stv {

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = dpp_i32<CTRL>(__double2loint(v));
  const int hi = dpp_i32<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// The value of lane k (0..3) of each quad of lanes, in every lane of the
// quad (k a constant once the caller's loops are unrolled).
__device__ __forceinline__ double quad_bcast_f64(double v, int k) {
  switch (k) {
    case 0: return dpp_f64<0x00>(v);   // quad_perm [0,0,0,0]
    case 1: return dpp_f64<0x55>(v);   // quad_perm [1,1,1,1]
    case 2: return dpp_f64<0xAA>(v);   // quad_perm [2,2,2,2]
    default: return dpp_f64<0xFF>(v);  // quad_perm [3,3,3,3]
  }
}

// Maximum over the 64 lanes, the same in every lane: within each row of 16
// lanes by partner exchanges (lane ^ 1, lane ^ 2, the mirrored quad of 8,
// the mirrored half of 16), then across the four rows by readlane.
__device__ __forceinline__ double wave_max_f64(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));    // quad_perm [1,0,3,2]
  v = fmax(v, dpp_f64<0x4E>(v));    // quad_perm [2,3,0,1]
  v = fmax(v, dpp_f64<0x141>(v));   // row_half_mirror
  v = fmax(v, dpp_f64<0x140>(v));   // row_mirror
  return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)),
              fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// Minimum over the 64 lanes, the same in every lane.
__device__ __forceinline__ int wave_min_i32(int v) {
  v = min(v, dpp_i32<0xB1>(v));
  v = min(v, dpp_i32<0x4E>(v));
  v = min(v, dpp_i32<0x141>(v));
  v = min(v, dpp_i32<0x140>(v));
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Maximum of unsigned 32-bit values over the 64 lanes, the same in every
// lane (partner exchanges inside rows of 16, then readlane across rows).
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)dpp_i32<0xB1>((int)v));
  v = max(v, (unsigned)dpp_i32<0x4E>((int)v));
  v = max(v, (unsigned)dpp_i32<0x141>((int)v));
  v = max(v, (unsigned)dpp_i32<0x140>((int)v));
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
  const unsigned b = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)v, 32);
  const unsigned d = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  return max(max(a, b), max(c, d));
}

// Pivot of one column with one candidate row per lane: the unused row of
// largest magnitude, the lowest such row on ties; -1 when no unused row holds
// a finite value.  Non-negative doubles order as their bit patterns, so the
// high words are compared first (a DPP max of 32-bit keys) and the low words
// only among the lanes that tie there.
__device__ __forceinline__ int pivot_lane(double x, bool cand) {
  const double ax = fabs(x);
  const unsigned hi = (unsigned)__double2hiint(ax);
  const unsigned key = (cand && ax == ax) ? hi + 1u : 0u;   // NaN and used rows: 0
  const unsigned kmax = wave_max_u32(key);
  if (kmax == 0u) return -1;
  uint64_t tied = __builtin_amdgcn_ballot_w64(key == kmax);
  if (tied & (tied - 1)) {
    const unsigned lo = (unsigned)__double2loint(ax);
    const unsigned lmax = wave_max_u32(key == kmax ? lo : 0u);
    tied = __builtin_amdgcn_ballot_w64(key == kmax && lo == lmax);
  }
  return (int)__builtin_ctzll(tied);
}

// 1 / x for a normal, nonzero x: the hardware reciprocal refined by two
// Newton steps (r <- r + r (1 - x r)), within an ulp or so of the rounded
// quotient; five dependent operations instead of the IEEE division sequence.
__device__ __forceinline__ double recip_f64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Orders the LDS accesses of one wavefront for the compiler: a store by one
// lane before the call is seen by loads of any lane after it (a wavefront's
// LDS instructions are processed in issue order, so no wait is needed).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace stv
