// dev_addsub.hpp -- work-group level addition / subtraction with a carry
// (borrow) scan, Section 5.1 (baddReg) and its mirror for subtraction.
#pragma once

#include "common.hpp"

namespace bi {

// One thread's run of Q limbs.  For addition each limb gives s = x + y with
// generate g = (s < x) and propagate p = (s == 0xffffffff); for subtraction
// d = x - y with g = (x < y) and p = (x == y).  The run summary composes the
// limbs low to high: G = g | (p & G), P = p & P (the carryBop of
// Section 5.1, without segment bits: one instance per work-group).
template <int Q, bool SUB>
struct LimbRun {
  uint32_t s[Q];
  uint64_t gm, pm;  // per-limb generate / propagate bit masks
  bool G, P;        // run summary

  // limb i of the run from operands x, y (past the end: transparent)
  __device__ __forceinline__ void set(int i, uint32_t x, uint32_t y, bool valid) {
    uint32_t r, g, p;
    if (SUB) { r = x - y; g = x < y; p = x == y; }
    else     { r = x + y; g = r < x; p = r == 0xffffffffu; }
    if (!valid) { r = 0; g = 0; p = 1; }
    s[i] = r;
    gm |= (uint64_t)g << i;
    pm |= (uint64_t)p << i;
  }

  __device__ __forceinline__ void start() { gm = 0; pm = 0; }

  // run summary from the per-limb bits, composed low to high
  __device__ __forceinline__ void finish() {
    bool Gs = false, Ps = true;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const bool g = (gm >> i) & 1u, p = (pm >> i) & 1u;
      Gs = g | (p & Gs);
      Ps = p & Ps;
    }
    G = Gs; P = Ps & !Gs;
  }

  __device__ __forceinline__ void build(const uint32_t (&x)[Q], const uint32_t (&y)[Q], int valid) {
    start();
#pragma unroll
    for (int i = 0; i < Q; ++i) set(i, x[i], y[i], i < valid);
    finish();
  }

  // apply the carry entering the run; returns the carry leaving it
  __device__ __forceinline__ uint32_t apply(uint32_t c) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      s[i] = SUB ? s[i] - c : s[i] + c;
      c = (uint32_t)(((gm >> i) & 1u) | (((pm >> i) & 1u) & c));
    }
    return c;
  }
};

// out[0..n) = X + Y (+cin), or X - Y (-cin), where X(j), Y(j) return limb j
// (j < n).  The whole work-group takes part; any n >= 0 works (rounds of
// blockDim*Q limbs, carry chained between rounds).  Returns the carry
// (borrow) out of limb n-1 in every thread.  out may alias the storage that
// X or Y read, limb for limb.
//
// SPARSE: out aliases X's storage and most Y limbs are zero; a limb is only
// stored when its value changes (saves rewriting the whole array).
// top (LDS, nullable): raised by atomicMax to 1 + the index of the highest
// nonzero result limb (the caller zeroes it before the call).
template <int Q, bool SUB, class FX, class FY, bool SPARSE = false>
__device__ __forceinline__ uint32_t wg_addsub(uint32_t* out, int n, FX X, FY Y, uint32_t cin, uint32_t* scratch,
                                              uint32_t* top = nullptr) {
  constexpr bool out_differs = false;
  const int T = blockDim.x;
  uint32_t carry = cin;
  for (int base = 0; base < n; base += T * Q) {
    const int j0 = base + threadIdx.x * Q;
    const int valid = min(Q, max(0, n - j0));
    uint32_t x[Q], y[Q];
    // limb indices clamped, values masked: no branch around the loads
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int jj = min(j0 + i, n - 1);
      const uint32_t xv = X(jj), yv = Y(jj);
      x[i] = (i < valid) ? xv : 0u;
      y[i] = (i < valid) ? yv : 0u;
    }
    LimbRun<Q, SUB> run;
    run.build(x, y, valid);
    uint32_t cout;
    const uint32_t c = wg_carry_scan(run.G, run.P, carry, scratch, &cout);
    run.apply(c);
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (i < valid && (!SPARSE || run.s[i] != x[i] || out_differs)) out[j0 + i] = run.s[i];
    if (top) {
      int m = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) m = (i < valid && run.s[i] != 0u) ? j0 + i + 1 : m;
      if (m) atomicMax(top, (uint32_t)m);
    }
    carry = cout;
    __syncthreads();
  }
  return carry;
}

}  // namespace bi
