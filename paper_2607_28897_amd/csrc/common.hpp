// common.hpp -- shared host and device helpers of the batched big-integer
// library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bigint_rocm.h"

typedef int v4i __attribute__((ext_vector_type(4)));

namespace bi {

// ---------------------------------------------------------------------------
// Host-side error plumbing
// ---------------------------------------------------------------------------
void set_hip_error(hipError_t e);

#define BI_HIP(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      ::bi::set_hip_error(e_);                                              \
      return BIGINT_EHIP;                                                   \
    }                                                                       \
  } while (0)

#define BI_LAUNCH_CHECK()                                                   \
  do {                                                                      \
    hipError_t e_ = hipGetLastError();                                      \
    if (e_ != hipSuccess) {                                                 \
      ::bi::set_hip_error(e_);                                              \
      return BIGINT_EHIP;                                                   \
    }                                                                       \
  } while (0)

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
__device__ __forceinline__ int num_waves() { return blockDim.x >> 6; }

// Floor / ceiling division of a (possibly negative) int by a positive int.
__device__ __forceinline__ int floor_div(int a, int b) {
  int q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}
__device__ __forceinline__ int ceil_div(int a, int b) { return -floor_div(-a, b); }

// Carry (or borrow) resolution over the 64 lanes of a wave.
//
// Each lane summarises a contiguous run of limbs by (g, p): g = the run emits
// a carry when none enters, p = the run passes an entering carry through
// (g and p are never both set).  This is the carry operator of Section 5.1
// (the pair (overflow, all-ones) combined by an associative operator and
// exclusively scanned).  On a wave the scan is one 64-bit integer addition
// of the ballot masks: with A = G|P and carry-in c, bit i of (A + G + c) ^ A
// ^ G is exactly the carry entering lane i, because a lane with g behaves
// like the bit pair (1,1), p like (1,0) and neither like (0,0).
struct WaveCarry {
  uint64_t G, P;
};

__device__ __forceinline__ WaveCarry wave_carry_masks(bool g, bool p) {
  WaveCarry w;
  w.G = __ballot(g);
  w.P = __ballot(p);
  return w;
}

// Carry into this lane given the carry c entering lane 0 of the wave.
__device__ __forceinline__ uint32_t wave_carry_in(const WaveCarry& w, uint32_t c) {
  const uint64_t A = w.G | w.P;
  const uint64_t S = A + w.G + (uint64_t)c;
  const uint64_t Cin = S ^ A ^ w.G;
  return (uint32_t)((Cin >> lane_id()) & 1ull);
}

// Carry leaving lane 63 given carry-in c.
__device__ __forceinline__ uint32_t wave_carry_out(const WaveCarry& w, uint32_t c) {
  const uint64_t A = w.G | w.P;
  const uint64_t s1 = A + w.G;
  const uint32_t o1 = s1 < A;             // overflow of A + G
  const uint64_t s2 = s1 + (uint64_t)c;
  const uint32_t o2 = s2 < s1;            // overflow of + c
  return o1 | o2;
}

// Work-group wide exclusive carry scan.  Every thread passes the (g, p)
// summary of its own limb run; returns the carry entering that run.  cin is
// the carry entering the whole work-group range.  `scratch` is >= 16 u32 of
// LDS; the function synchronises the work-group twice and leaves scratch
// free for reuse on return.  *cout (optional, all threads) = carry leaving
// the last thread.
__device__ __forceinline__ uint32_t wg_carry_scan(bool g, bool p, uint32_t cin,
                                                  uint32_t* scratch,
                                                  uint32_t* cout) {
  const WaveCarry w = wave_carry_masks(g, p);
  const int wid = wave_id(), nw = num_waves();
  // wave summary for the work-group level: generate with carry-in 0,
  // propagate = every lane propagates
  const uint32_t gw = wave_carry_out(w, 0);
  const uint32_t pw = (w.P == ~0ull);
  if (lane_id() == 0) scratch[wid] = gw | (pw << 1);
  __syncthreads();
  uint32_t c = cin;
  for (int k = 0; k < wid; ++k) {
    const uint32_t s = scratch[k];
    c = (s & 1u) | ((s >> 1) & c);
  }
  if (cout) {
    uint32_t t = c;
    for (int k = wid; k < nw; ++k) {
      const uint32_t s = scratch[k];
      t = (s & 1u) | ((s >> 1) & t);
    }
    *cout = t;
  }
  const uint32_t r = wave_carry_in(w, c);
  __syncthreads();
  return r;
}

// Bits [7k, 7k+7) of the n-limb integer a (0 outside): the k-th 7-bit digit.
__device__ __forceinline__ uint32_t digit7(const uint32_t* __restrict__ a, int n, int k) {
  const int bit = 7 * k;
  const int l = bit >> 5, s = bit & 31;
  if (k < 0 || l >= n) return 0;
  uint32_t v = a[l] >> s;
  if (s > 25 && l + 1 < n) v |= a[l + 1] << (32 - s);
  return v & 127u;
}

}  // namespace bi
