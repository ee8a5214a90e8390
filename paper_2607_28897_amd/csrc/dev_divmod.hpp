// dev_divmod.hpp -- division through the whole shifted inverse (Section 5.3).
//
// For a divisor v with k1 significant limbs (B = 2^32) and a dividend u with
// h significant limbs, the quotient is read off w ~ B^h / v:
// q~ = floor(u w / B^h) is within a few units of floor(u / v), and the signed
// remainder u - q~ v, reduced into [0, v) by adding or subtracting v, fixes
// it.  w is grown by Newton steps in the integral domain, the paper's `step`
// (Section 5.3, Fig. bdiv-F-code) with both of its branches: with
// e = B^c - V w (the signed powDiff, V the divisor's top limbs),
//     w' = w B^m + floor(w e / B^(c-m))      if e > 0
//     w' = w B^m - ceil(w |e| / B^(c-m))     if e <= 0
// (the ceiling: the truncated quotient plus one unless the dropped limbs are
// all zero -- nullUpToInd and baddOne).  If w is within eta units of B^c / V,
// w' is within eta^2 B^(m-c+t) + 1 units of B^(c+m) / V; one guard limb
// (m <= c - t - 1) keeps eta below 2 at every scale with no exact fix-up, so
// the whole procedure takes no correction step before the quotient's.  The
// starting value is the exact floor(B^(t0+2) / V0) of the top t0 = min(k1, 4)
// limbs of v, within one unit of B^(k1+2) / v.  Multiplications run on the
// MFMA-split multiply at their operands' actual lengths (low products where
// only limbs below a bound are needed); linear operations (precision,
// shifts, additions, comparisons) run on the whole work-group.  Division by
// a one-limb divisor is a short division.
#pragma once

#include "common.hpp"
#include "dev_addsub.hpp"
#include "dev_mul_mfma.hpp"

namespace bi {
namespace div {

constexpr int kP = 4;   // strips per band of the multiplications
constexpr int kDW = 8;  // digit width of the multiplications
constexpr int kMaxAdjust = 64;  // cap on the exact fix-up's rounds (the inverse diagnostic)
constexpr int kGuard = 2;       // divisor limbs kept beyond the precision of a Newton step

// LDS words used by the division itself (besides the multiply's area)
struct Shared {
  uint32_t red[4];      // reductions
  uint32_t scan[32];    // carry-scan scratch
  uint32_t w0[4];       // initial estimate (one thread)
  int early_cur, early_lw;  // scale and length of w after the one-wave steps
  uint32_t failed;      // a bounded loop hit its bound, or an estimate left its error bound (never expected)
};

// ---- work-group linear operations on global limb arrays ------------------------

// The loops below are unrolled with unconditional loads so that each thread
// keeps several global loads in flight (one work-group per division cannot
// hide memory latency with other work-groups).

__device__ __forceinline__ void wg_fill(uint32_t* x, int n, uint32_t v) {
#pragma unroll 4
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = v;
  __syncthreads();
}

__device__ __forceinline__ void wg_copy(uint32_t* dst, const uint32_t* src, int n) {
#pragma unroll 8
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
}

// dst[0..n) = src[s .. s+n) (limbs past ns read as 0); dst must not overlap src
__device__ __forceinline__ void wg_shr_copy(uint32_t* dst, int n, const uint32_t* src, int ns, int s) {
#pragma unroll 8
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int j = i + s;
    const uint32_t v = ns > 0 ? src[min(j, ns - 1)] : 0u;
    dst[i] = j < ns ? v : 0u;
  }
  __syncthreads();
}

// number of significant limbs of x[0..n)
// Short operands (n <= 64 * kWaveRounds limbs) are reduced inside every wave
// from per-round ballots (limb 64 r + lane in round r), which needs no LDS
// reduction and no barrier between waves; one closing barrier keeps a later
// in-place write from overtaking a slower wave's reads.
constexpr int kWaveRounds = 2;

__device__ __forceinline__ int wg_prec(const uint32_t* x, int n, Shared* sh) {
  if (n <= 64 * kWaveRounds) {
    int top = 0;
    uint64_t mk[kWaveRounds];
#pragma unroll
    for (int r = 0; r < kWaveRounds; ++r) {
      const int i = 64 * r + lane_id();
      const uint32_t v = n > 0 ? x[min(i, n - 1)] : 0u;
      mk[r] = __ballot(i < n && v != 0u);
    }
#pragma unroll
    for (int r = kWaveRounds - 1; r >= 0; --r)
      if (top == 0 && mk[r] != 0ull) top = 64 * r + 64 - __clzll(mk[r]);
    __syncthreads();
    return top;
  }
  if (threadIdx.x == 0) sh->red[0] = 0;
  __syncthreads();
  int m = 0;
#pragma unroll 8
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = x[i] != 0u ? i + 1 : m;
  if (m) atomicMax(&sh->red[0], (uint32_t)m);
  __syncthreads();
  const int r = (int)sh->red[0];
  __syncthreads();
  return r;
}

// the significant limbs of x[0..nx) and of y[0..ny) in one pass (the loads
// of both arrays in flight together, one reduction)
__device__ __forceinline__ void wg_prec2(const uint32_t* x, int nx, const uint32_t* y, int ny,
                                         Shared* sh, int* px, int* py) {
  if (max(nx, ny) <= 64 * kWaveRounds) {
    *px = wg_prec(x, nx, sh);
    *py = wg_prec(y, ny, sh);
    return;
  }
  // the usual case first: a nonzero limb among the top 64 of each settles
  // its precision with one load per lane (every wave the same ballots)
  {
    const int i = lane_id();
    const uint32_t a = nx > i ? x[nx - 1 - i] : 0u, b = ny > i ? y[ny - 1 - i] : 0u;
    const uint64_t ma = __ballot(a != 0u), mb = __ballot(b != 0u);
    if (ma != 0ull && mb != 0ull) {
      *px = nx - (__ffsll((long long)ma) - 1);
      *py = ny - (__ffsll((long long)mb) - 1);
      return;
    }
  }
  if (threadIdx.x == 0) { sh->red[0] = 0; sh->red[1] = 0; }
  __syncthreads();
  int mx = 0, my = 0;
  const int n = max(nx, ny);
#pragma unroll 8
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const uint32_t a = nx > 0 ? x[min(i, nx - 1)] : 0u, b = ny > 0 ? y[min(i, ny - 1)] : 0u;
    mx = (i < nx && a != 0u) ? i + 1 : mx;
    my = (i < ny && b != 0u) ? i + 1 : my;
  }
  if (mx) atomicMax(&sh->red[0], (uint32_t)mx);
  if (my) atomicMax(&sh->red[1], (uint32_t)my);
  __syncthreads();
  *px = (int)sh->red[0];
  *py = (int)sh->red[1];
  __syncthreads();
}

// sign of x - y over n limbs (both zero-extended to n), and whether x is 0,
// in one pass
struct Cmp { int sign; bool xzero; };

// x - y over n <= 64 * kWaveRounds limbs inside every wave: sign of the
// highest differing limb, and whether x is zero
__device__ __forceinline__ Cmp wave_cmp_z(const uint32_t* x, int nx, const uint32_t* y, int ny,
                                          int n) {
  uint32_t av[kWaveRounds], bv[kWaveRounds];
  uint64_t dk[kWaveRounds], zk = 0;
#pragma unroll
  for (int r = 0; r < kWaveRounds; ++r) {
    const int i = 64 * r + lane_id();
    const uint32_t a = nx > 0 ? x[min(i, nx - 1)] : 0u, b = ny > 0 ? y[min(i, ny - 1)] : 0u;
    av[r] = (i < nx && i < n) ? a : 0u;
    bv[r] = (i < ny && i < n) ? b : 0u;
    dk[r] = __ballot(av[r] != bv[r]);
    zk |= __ballot(av[r] != 0u);
  }
  Cmp res{0, zk == 0ull};
  bool found = false;
#pragma unroll
  for (int r = kWaveRounds - 1; r >= 0; --r) {
    if (!found && dk[r] != 0ull) {
      const int bit = 63 - __clzll(dk[r]);
      const uint32_t a = __shfl(av[r], bit), b = __shfl(bv[r], bit);
      res.sign = a > b ? 1 : -1;
      found = true;
    }
  }
  __syncthreads();
  return res;
}

__device__ __forceinline__ Cmp wg_cmp_z(const uint32_t* x, int nx, const uint32_t* y, int ny, int n,
                                        Shared* sh) {
  if (n <= 64 * kWaveRounds) return wave_cmp_z(x, nx, y, ny, n);
  if (threadIdx.x == 0) { sh->red[1] = 0; sh->red[2] = 0; }
  __syncthreads();
  int m = 0, z = 0;
#pragma unroll 8
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const uint32_t a = nx > 0 ? x[min(i, nx - 1)] : 0u, b = ny > 0 ? y[min(i, ny - 1)] : 0u;
    const uint32_t av = i < nx ? a : 0u, bv = i < ny ? b : 0u;
    m = av != bv ? i + 1 : m;
    z = av != 0u ? 1 : z;
  }
  if (m) atomicMax(&sh->red[1], (uint32_t)m);
  if (z) sh->red[2] = 1u;
  __syncthreads();
  const int top = (int)sh->red[1];
  Cmp r{0, sh->red[2] == 0u};
  if (top) {
    const uint32_t a = top - 1 < nx ? x[top - 1] : 0u, b = top - 1 < ny ? y[top - 1] : 0u;
    r.sign = a > b ? 1 : -1;
  }
  __syncthreads();
  return r;
}

// sign of x - y over n limbs (both zero-extended to n)
__device__ __forceinline__ int wg_cmp(const uint32_t* x, int nx, const uint32_t* y, int ny, int n,
                                      Shared* sh) {
  if (n <= 64 * kWaveRounds) return wave_cmp_z(x, nx, y, ny, n).sign;
  if (threadIdx.x == 0) sh->red[1] = 0;
  __syncthreads();
  int m = 0;
#pragma unroll 8
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const uint32_t a = nx > 0 ? x[min(i, nx - 1)] : 0u, b = ny > 0 ? y[min(i, ny - 1)] : 0u;
    const uint32_t av = i < nx ? a : 0u, bv = i < ny ? b : 0u;
    m = av != bv ? i + 1 : m;
  }
  if (m) atomicMax(&sh->red[1], (uint32_t)m);
  __syncthreads();
  const int top = (int)sh->red[1];
  int r = 0;
  if (top) {
    const uint32_t a = top - 1 < nx ? x[top - 1] : 0u, b = top - 1 < ny ? y[top - 1] : 0u;
    r = a > b ? 1 : -1;
  }
  __syncthreads();
  return r;
}

// addition / subtraction for the division on the whole work-group.  (Running
// short ranges inside every wave instead, with two barriers, raised the
// kernel's register spills from 180 to 388 bytes per lane and made divisions
// 9% slower.)
template <bool SUB, class FX, class FY>
__device__ __forceinline__ uint32_t div_addsub(uint32_t* out, int n, FX X, FY Y, Shared* sh,
                                               uint32_t* top = nullptr, uint32_t cin = 0u) {
  return wg_addsub<16, SUB>(out, n, X, Y, cin, sh->scan, top);
}

// dst[0..n) = x + y (or x - y), operands zero-extended; returns carry/borrow
template <bool SUB>
__device__ __forceinline__ uint32_t wg_arith(uint32_t* dst, int n, const uint32_t* x, int nx,
                                             const uint32_t* y, int ny, Shared* sh) {
  auto X = [&](int j) -> uint32_t { return (j < nx) ? x[min(j, nx - 1)] : 0u; };
  auto Y = [&](int j) -> uint32_t { return (j < ny) ? y[min(j, ny - 1)] : 0u; };
  return div_addsub<SUB>(dst, n, X, Y, sh);
}

// dst[0..n) = x +/- small (a one-limb value), x zero-extended
template <bool SUB>
__device__ __forceinline__ uint32_t wg_arith1(uint32_t* dst, int n, const uint32_t* x, int nx,
                                              uint32_t small, Shared* sh) {
  auto X = [&](int j) -> uint32_t { return (j < nx) ? x[min(j, nx - 1)] : 0u; };
  auto Y = [&](int j) -> uint32_t { return j == 0 ? small : 0u; };
  return div_addsub<SUB>(dst, n, X, Y, sh);
}

constexpr int kSmallMul = 64;  // operands up to this many limbs: column-sum product
// LDS bytes of the column-sum product (both operands staged)
constexpr size_t kSmallMulLds = (size_t)2 * kSmallMul * 4;

// Lane l holds the sums of product columns k = l + 64 g (g < H) as
// C_k = s_k + 2^64 c_k.  Writes limbs [0, n) (n <= 64 H) of sum_k C_k B^k to
// dst: limb k receives lo32(s_k) + hi32(s_(k-1)) + c_(k-2) (< 3 * 2^32), whose
// overflow (at most 2) goes one limb up through wave-level carry scans over
// limbs 0..63, 64..127, ...
template <int H>
__device__ __forceinline__ void wave_cols_to_limbs(const uint64_t (&s)[H], const uint32_t (&c)[H],
                                                   uint32_t* dst, int n) {
  const int l = lane_id();
  // neighbours: column k-1 and k-2 (lane l-1 / l-2 of the same group, or of
  // the group below across the lane-0 boundary)
  const int l1 = (l + 63) & 63, l2 = (l + 62) & 63;
  uint32_t sh[H], cc[H];
#pragma unroll
  for (int g = 0; g < H; ++g) {
    sh[g] = __shfl((uint32_t)(s[g] >> 32), l1);
    cc[g] = __shfl(c[g], l2);
  }
  uint32_t tl[H], th[H];
#pragma unroll
  for (int g = 0; g < H; ++g) {
    const int k = l + 64 * g;
    const uint32_t hi1 = k >= 1 ? (l >= 1 ? sh[g] : sh[g > 0 ? g - 1 : 0]) : 0u;
    const uint32_t cc2 = k >= 2 ? (l >= 2 ? cc[g] : cc[g > 0 ? g - 1 : 0]) : 0u;
    const uint64_t t = (uint64_t)(uint32_t)s[g] + hi1 + cc2;
    tl[g] = (uint32_t)t;
    th[g] = (uint32_t)(t >> 32);
  }
  // limb k = tl_k + th_(k-1), carries rippling up
  uint32_t tt[H];
#pragma unroll
  for (int g = 0; g < H; ++g) tt[g] = __shfl(th[g], l1);
  uint32_t carry = 0u;
#pragma unroll
  for (int g = 0; g < H; ++g) {
    const int k = l + 64 * g;
    const uint32_t y = k >= 1 ? (l >= 1 ? tt[g] : tt[g > 0 ? g - 1 : 0]) : 0u;
    const uint32_t x = tl[g];
    const uint32_t r = x + y;
    const bool gen = r < x, p = r == 0xffffffffu;
    const WaveCarry w = wave_carry_masks(gen, p);
    const uint32_t ci = wave_carry_in(w, carry);
    carry = wave_carry_out(w, carry);
    if (k < n) dst[k] = r + ci;
  }
}

// dst[0 .. n) = a * b mod B^n with n = na + nb (nout < 0) or min(nout, na + nb),
// for 1 <= na, nb <= kSmallMul, on wave 0 alone (the other waves wait at the
// closing barrier).  The MFMA multiply's fixed steps (digit staging, prefix
// sums, band scheduling, barriers) cost several microseconds even for a few
// limbs, which the early Newton steps would pay twice per step.  Wave 0
// stages both operands in LDS; lane l forms columns k = l and l + 64,
// C_k = sum a_i b_(k-i) of 32 x 32-bit products, as a 64-bit sum s_k plus a
// count c_k of its carries.  Limb k of the product then receives
// lo32(s_k) + hi32(s_(k-1)) + c_(k-2) (< 3 * 2^32), whose overflow (at most 2)
// goes one limb up through two wave-level carry scans (limbs 0..63, then
// 64..127).
__device__ inline void wg_mul_small(uint32_t* dst, const uint32_t* a, int na, const uint32_t* b,
                                    int nb, char* smem, int nout) {
  if (wave_id() == 0) {
    uint32_t* sa = reinterpret_cast<uint32_t*>(smem);
    uint32_t* sb = sa + kSmallMul;
    const int l = lane_id();
    const int K = na + nb;
    const int n = nout < 0 ? K : min(nout, K);
    if (l < na) sa[l] = a[l];
    if (l < nb) sb[l] = b[l];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint64_t s[2];
    uint32_t c[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = l + 64 * h;
      uint64_t sum = 0;
      uint32_t cnt = 0;
      const int lo = max(0, k - nb + 1), hi = min(k, na - 1);
      for (int i = lo; i <= hi; ++i) {
        const uint64_t t = (uint64_t)sa[i] * sb[k - i] + sum;
        cnt += t < sum;
        sum = t;
      }
      s[h] = sum;
      c[h] = cnt;
    }
    wave_cols_to_limbs<2>(s, c, dst, n);
  }
  __syncthreads();
}

// adjust (nullable): adjust[3] += the int8 multiply-accumulates of the MFMA
// products (digit pairs (i, j) of the computed strips: i + j from 256 times
// the first computed strip up to 256 times their end); the column-sum
// products run on the vector ALU and add none.
__host__ __device__ inline int64_t tri(int64_t x) { return x > 0 ? x * (x + 1) / 2 : 0; }

// digit pairs (i, j) in [0, Na) x [0, Nb) with i + j < lim, by inclusion and exclusion
__host__ __device__ inline int64_t pairs_below(int64_t Na, int64_t Nb, int64_t lim) {
  return tri(lim) - tri(lim - Na) - tri(lim - Nb) + tri(lim - Na - Nb);
}

__host__ __device__ inline int64_t mfma_pairs(int na, int nb, int nout, int nlo) {
  const int64_t Na = mfma::ndigits_w<kDW>(na), Nb = mfma::ndigits_w<kDW>(nb);
  const int64_t K = Na + Nb - 1;
  const int64_t lim = nout < 0 ? K : min(K, (int64_t)mfma::kStrip *
                                             ((nout + mfma::strip_limbs<kDW>() - 1) / mfma::strip_limbs<kDW>()));
  const int64_t lo = min(lim, (int64_t)mfma::kStrip * kP * mfma::high_band<kDW>(nlo, kP));
  return pairs_below(Na, Nb, lim) - pairs_below(Na, Nb, lo);
}

// dst[0 .. nout) = a * b mod B^nout (nout < 0: all na+nb limbs; dst must not
// overlap a, b): small operands by column sums, the rest on the MFMA-split
// multiply.  nlo > 0: only the limbs from nlo up are needed, and the MFMA
// multiply may skip the strips below (dst[nlo ..) is then floor(a b / B^nlo)
// or one less).  Returns true when every limb of dst is exact.  One
// out-of-line copy serves every call site of the division, so the kernel's
// code stays small enough for the instruction cache.
__device__ __noinline__ bool wg_mul(uint32_t* dst, const uint32_t* a, int na, const uint32_t* b,
                                    int nb, char* smem, int nout, int64_t* adjust, int nlo = 0) {
  if (na <= kSmallMul && nb <= kSmallMul) {
    wg_mul_small(dst, a, na, b, nb, smem, nout);
    return true;
  }
  if (adjust) adjust[3] += mfma_pairs(na, nb, nout, nlo);
  mfma::wg_mul_mfma<kDW, kP>(dst, nullptr, a, na, b, nb, smem, nout, nlo);
  return mfma::high_band<kDW>(nlo, kP) == 0;
}

// ---- the first Newton steps on one wave ---------------------------------------------
// While every operand of a step fits in 128 limbs (two per lane), wave 0
// runs the step alone out of LDS: column-sum products, ballot carry scans,
// no work-group barrier and no global round trip, while the other waves
// wait at one barrier.  (On the whole work-group each such step took
// 10-12 us, nearly all of it the fixed latency of a dozen passes and
// barriers.  Four limbs per lane, which takes one more step onto the wave,
// measured 1% slower: one wave's serial column sums then cost as much as
// the work-group's step.)
constexpr int kWaveGroups = 2;                             // limbs per lane
constexpr int kWaveLimbs = 64 * kWaveGroups;
constexpr int kEarlyArr = kWaveLimbs + 8;                  // limbs per LDS array
constexpr size_t kEarlyLds = (size_t)5 * kEarlyArr * 4;   // w, new w, e, w e, V

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// dst[0 .. n) = a * b mod B^n for n <= kWaveLimbs, operands and result in
// LDS (dst must not overlap them); lane l forms columns l + 64 g
__device__ inline void wave_mul_lds(uint32_t* dst, const uint32_t* sa, int na, const uint32_t* sb,
                                    int nb, int n) {
  const int l = lane_id();
  uint64_t s[kWaveGroups];
  uint32_t c[kWaveGroups];
#pragma unroll
  for (int g = 0; g < kWaveGroups; ++g) {
    const int k = l + 64 * g;
    uint64_t sum = 0;
    uint32_t cnt = 0;
    const int lo = max(0, k - nb + 1), hi = min(min(k, na - 1), k < n ? k : -1);
    for (int i = lo; i <= hi; ++i) {
      const uint64_t t = (uint64_t)sa[i] * sb[k - i] + sum;
      cnt += t < sum;
      sum = t;
    }
    s[g] = sum;
    c[g] = cnt;
  }
  wave_cols_to_limbs<kWaveGroups>(s, c, dst, n);
  wave_lds_sync();
}

// dst[j] = X(j) + Y(j) (+ cin) or X(j) - Y(j) (- cin) for j < n <= kWaveLimbs
// on one wave (every X, Y read before dst is written); returns the number
// of significant limbs of the result
template <bool SUB, class FX, class FY>
__device__ inline int wave_addsub_w(uint32_t* dst, int n, FX X, FY Y, uint32_t cin) {
  const int l = lane_id();
  uint32_t xs[kWaveGroups], ys[kWaveGroups];
#pragma unroll
  for (int g = 0; g < kWaveGroups; ++g) {
    const int j = l + 64 * g;
    xs[g] = j < n ? X(j) : 0u;
    ys[g] = j < n ? Y(j) : 0u;
  }
  wave_lds_sync();
  uint32_t carry = cin;
  int top = 0;
#pragma unroll
  for (int g = 0; g < kWaveGroups; ++g) {
    const int j = l + 64 * g;
    const bool in = j < n;
    const uint32_t x = xs[g], y = ys[g];
    const uint32_t r = SUB ? x - y : x + y;
    const bool gen = in && (SUB ? x < y : r < x);
    const bool p = in && (SUB ? x == y : r == 0xffffffffu);
    const WaveCarry w = wave_carry_masks(gen, p);
    const uint32_t ci = wave_carry_in(w, carry);
    carry = wave_carry_out(w, carry);
    const uint32_t res = SUB ? r - ci : r + ci;
    if (in) dst[j] = res;
    const uint64_t nz = __ballot(in && res != 0u);
    if (nz) top = 64 * g + 64 - __clzll(nz);
  }
  wave_lds_sync();
  return top;
}

// The Newton steps of shifted_inverse (same formulas, same products, all
// exact) from scale cur while each fits one wave; wave 0 only.  w: lw limbs
// in global memory on entry and on return; smem: kEarlyLds bytes of LDS.
// Updates cur and lw; failed is set if an estimate leaves its error bound.
__device__ inline void wave_newton_early(const uint32_t* v, int k1, int h, uint32_t* W, char* smem,
                                         int64_t* adjust, int& cur, int& lw, bool& failed) {
  uint32_t* sW = reinterpret_cast<uint32_t*>(smem);
  uint32_t* sU = sW + kEarlyArr;
  uint32_t* sE = sU + kEarlyArr;
  uint32_t* sT = sE + kEarlyArr;
  uint32_t* sV = sT + kEarlyArr;
  const int l = lane_id();
#pragma unroll
  for (int g = 0; g < kWaveGroups; ++g) {
    const int j = l + 64 * g;
    sW[j] = j < lw ? W[j] : 0u;
  }
  wave_lds_sync();
  while (cur < h) {
    const int m = min(h - cur, cur - k1 - 1);
    const int t = min(k1, cur + m - k1 + 1 + kGuard);
    const int sdrop = k1 - t;
    const int c = cur - sdrop;
    const int le = t + 2;
    const int sd = max(0, min(le - 1, c - m - 1 - lw));
    const int ly = lw + le - sd;
    const int lnew = lw + m + 1;
    if (le > kWaveLimbs || ly > kWaveLimbs || lnew > kWaveLimbs) break;
#pragma unroll
    for (int g = 0; g < kWaveGroups; ++g) {
      const int j = l + 64 * g;
      if (j < t) sV[j] = v[sdrop + j];
    }
    wave_lds_sync();
    // powDiff from the low product, as on the work-group
    wave_mul_lds(sE, sV, t, sW, lw, le);
    const uint32_t top = __builtin_amdgcn_readfirstlane(sE[le - 1]);
    const bool neg = top == 0u;
    if (!neg) {
      if (top != 0xffffffffu) { failed = true; break; }
      wave_addsub_w<true>(sE, le, [](int) -> uint32_t { return 0u; },
                           [&](int j) -> uint32_t { return sE[j]; }, 0u);
    }
    if (adjust) {
      adjust[0] += 1;
      adjust[1] += neg ? 1 : 0;
    }
    // step (the whole product w |e|: the ceiling's dropped-limb test is exact)
    wave_mul_lds(sT, sW, lw, sE + sd, le - sd, ly);
    const int sy = c - m - sd;
    uint32_t cin = 0u;
    if (neg) {
      const int nlow = min(sy, ly);
      bool nz = false;
#pragma unroll
      for (int g = 0; g < kWaveGroups; ++g) nz |= l + 64 * g < nlow && sT[l + 64 * g] != 0u;
      cin = __ballot(nz) != 0ull ? 1u : 0u;
    }
    auto X = [&](int j) -> uint32_t { return (j >= m && j - m < lw) ? sW[j - m] : 0u; };
    auto Y = [&](int j) -> uint32_t { return j + sy < ly ? sT[j + sy] : 0u; };
    const int top2 = neg ? wave_addsub_w<true>(sU, lnew, X, Y, cin)
                         : wave_addsub_w<false>(sU, lnew, X, Y, 0u);
    uint32_t* tmp = sW;
    sW = sU;
    sU = tmp;
    lw = max(top2, 1);
    cur += m;
  }
#pragma unroll
  for (int g = 0; g < kWaveGroups; ++g) {
    const int j = l + 64 * g;
    if (j < lw) W[j] = sW[j];
  }
}

// ---- one-lane helper for the starting value ------------------------------------

// floor(B^(N+2) / V) for an N-limb V with a nonzero top limb (B = 2^32), by
// long division in base B (Knuth, TAOCP vol. 2, 4.3.1, Algorithm D):
// normalise V so its top bit is set, then four quotient limbs, each
// estimated from the top two remainder limbs and the divisor's top limb,
// corrected by the divisor's second limb and a final add-back.  N is a
// compile-time constant, so every limb array lives in registers.
template <int N>
__device__ inline unsigned __int128 seed_div(const uint32_t* v, int k1) {
  constexpr int M = 3;   // the dividend B^(N+2) has N + 3 limbs
  uint32_t vn[N], un[N + M + 1];
  const int sft = __clz(v[k1 - 1]);
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    const uint32_t hi = v[k1 - N + i];
    const uint32_t lo = i > 0 ? v[k1 - N + i - 1] : 0u;
    vn[i] = sft ? (hi << sft) | (lo >> (32 - sft)) : hi;
  }
#pragma unroll
  for (int i = 0; i < N + M + 1; ++i) un[i] = 0u;
  un[N + 2] = 1u << sft;
  uint32_t q[M + 1];
#pragma unroll
  for (int j = M; j >= 0; --j) {
    const uint64_t num = ((uint64_t)un[j + N] << 32) | un[j + N - 1];
    uint64_t qhat = num / vn[N - 1];
    uint64_t rhat = num - qhat * vn[N - 1];
    for (int k = 0; k < 2; ++k) {
      if (qhat >= (1ull << 32) || qhat * vn[N - 2] > ((rhat << 32) | un[j + N - 2])) {
        --qhat;
        rhat += vn[N - 1];
        if (rhat < (1ull << 32)) continue;
      }
      break;
    }
    // un[j .. j+N] -= qhat * vn
    int64_t borrow = 0;
    uint64_t carry = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const uint64_t p = qhat * vn[i] + carry;
      carry = p >> 32;
      const int64_t t = (int64_t)un[i + j] - (int64_t)(uint32_t)p + borrow;
      un[i + j] = (uint32_t)t;
      borrow = t >> 32;
    }
    const int64_t t = (int64_t)un[j + N] - (int64_t)carry + borrow;
    un[j + N] = (uint32_t)t;
    if (t < 0) {   // qhat was one too large: add V back
      --qhat;
      uint64_t c = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const uint64_t x = (uint64_t)un[i + j] + vn[i] + c;
        un[i + j] = (uint32_t)x;
        c = x >> 32;
      }
      un[j + N] += (uint32_t)c;
    }
    q[j] = (uint32_t)qhat;
  }
  unsigned __int128 w = 0;
#pragma unroll
  for (int j = M; j >= 0; --j) w = (w << 32) | q[j];
  return w;
}

// floor(B^(t0+2) / V) for the top t0 = min(k1, 4) limbs V of v (k1 >= 2):
// at most B^3 (97 bits)
__device__ inline unsigned __int128 seed_inverse(const uint32_t* v, int k1) {
  if (k1 >= 4) return seed_div<4>(v, k1);
  if (k1 == 3) return seed_div<3>(v, k1);
  return seed_div<2>(v, k1);
}

// ---- the division of one instance ----------------------------------------------

struct Bufs {
  uint32_t* W;   // w, capacity cw
  uint32_t* E;   // e, capacity ce
  uint32_t* T;   // products, capacity ct
  uint32_t* U2;  // second temporary (new w, remainder), capacity cw
  int cw, ce, ct;
};

__host__ __device__ inline size_t div_ws_limbs(int nu, int nv) {
  const int cw = nu + 8, ce = nv + 8, ct = 2 * nu + nv + 16;
  return (size_t)2 * cw + ce + ct;
}

__host__ __device__ inline Bufs carve_bufs(uint32_t* ws, int nu, int nv) {
  Bufs b;
  b.cw = nu + 8; b.ce = nv + 8; b.ct = 2 * nu + nv + 16;
  b.W = ws; b.U2 = b.W + b.cw; b.E = b.U2 + b.cw; b.T = b.E + b.ce;
  return b;
}

// Exact fix-up at scale c: given w (lw limbs, approximately floor(B^c / v)),
// make w = floor(B^c / v) and E = B^c - v w in [0, v).  Returns the new lw.
// adjust (nullable): diagnostic counters; adjust[1] += the unit steps of w.
__device__ inline int fixup(const uint32_t* v, int k1, int c, Bufs& bf, int lw, Shared* sh,
                            char* smem, int64_t* adjust) {
  // P = v * w
  const int lp = k1 + lw;
  const int le = max(k1 + 2, 2);
  bool neg = false;
  bool have_e = false;
  if (c >= le && lp > le) {
    // |e| = |B^c - P| is a few v at most, below B^(le-1): P mod B^le then
    // ends in limb 0 (P >= B^c, and P mod B^le = P - B^c) or in an all-ones
    // limb (P < B^c, e = -P mod B^le), so the low le limbs of P suffice.  Any
    // other top limb means a far estimate: the whole product below decides.
    wg_mul(bf.T, v, k1, bf.W, lw, smem, le, adjust);
    // every wave reads the same limb after the multiply's closing barrier
    const uint32_t top = __builtin_amdgcn_readfirstlane(bf.T[le - 1]);
    if (top == 0u) {
      neg = true;
      wg_copy(bf.E, bf.T, le);
      have_e = true;
    } else if (top == 0xffffffffu) {
      neg = false;
      auto X = [&](int) -> uint32_t { return 0u; };
      auto Y = [&](int j) -> uint32_t { return bf.T[j]; };
      div_addsub<true>(bf.E, le, X, Y, sh);
      have_e = true;
    }
  }
  if (!have_e) {
    wg_mul(bf.T, v, k1, bf.W, lw, smem, -1, adjust);
    // sign: P >= B^c  <=>  some limb at index >= c is nonzero
    const int pp = wg_prec(bf.T, lp, sh);
    if (pp <= c) {
      // e = B^c - P (P < B^c): the low c limbs of 0 - P; it is < few v
      neg = false;
      auto X = [&](int) -> uint32_t { return 0u; };
      auto Y = [&](int j) -> uint32_t { return j < lp ? bf.T[j] : 0u; };
      div_addsub<true>(bf.T, min(c, lp), X, Y, sh);  // in place
      // limbs [min(c,lp), c) of 0 - P are all ones only if P == 0, which w >= 1 rules out
      wg_shr_copy(bf.E, le, bf.T, min(c, lp), 0);
      if (c > lp) {
        // B^c - P with P < B^lp <= B^(c-1): e would be >= B^(c-1) -- far from w
        // exact; keep it exact anyway by filling the all-ones limbs
        for (int i = threadIdx.x; i < le; i += blockDim.x)
          if (i >= lp && i < c) bf.E[i] = 0xffffffffu;
        __syncthreads();
      }
    } else {
      // e = -(P - B^c)
      neg = true;
      wg_arith1<true>(bf.T + c, lp - c, bf.T + c, lp - c, 1u, sh);
      wg_shr_copy(bf.E, le, bf.T, lp, 0);
    }
  }
  int adj = 0;
  if (neg) {
    // the usual cases in one pass: e = 0 (w is exact) or -v <= e < 0 (one
    // step down: w -= 1, e = v - |e|)
    const Cmp cz = wg_cmp_z(bf.E, le, v, k1, le, sh);
    if (cz.xzero) return lw;   // v w = B^c: w is exact and e = 0
    if (cz.sign <= 0) {
      wg_arith1<true>(bf.W, lw, bf.W, lw, 1u, sh);
      wg_arith<true>(bf.E, le, v, k1, bf.E, le, sh);
      neg = false;
      ++adj;
      if (adjust) adjust[1] += adj;
      return lw;
    }
  }
  // while e < 0: w -= 1, e += v   (a correct estimate needs at most a few
  // rounds; the cap only guarantees that every wave terminates)
  while (neg && adj < kMaxAdjust) {
    wg_arith1<true>(bf.W, lw, bf.W, lw, 1u, sh);
    // |e| vs v
    const int s = wg_cmp(bf.E, le, v, k1, le, sh);
    if (s > 0) {
      wg_arith<true>(bf.E, le, bf.E, le, v, k1, sh);   // |e| - v, still negative
    } else {
      wg_arith<true>(bf.E, le, v, k1, bf.E, le, sh);   // v - |e| >= 0
      neg = false;
    }
    ++adj;
  }
  // while e >= v: w += 1, e -= v
  while (adj < kMaxAdjust) {
    const int s = wg_cmp(bf.E, le, v, k1, le, sh);
    if (s < 0) break;
    wg_arith<true>(bf.E, le, bf.E, le, v, k1, sh);
    const uint32_t c2 = wg_arith1<false>(bf.W, lw, bf.W, lw, 1u, sh);
    if (c2) {  // w grew by one limb
      if (threadIdx.x == 0) bf.W[lw] = 1u;
      __syncthreads();
      ++lw;
    }
    ++adj;
  }
  if (adjust) adjust[1] += adj;
  if (adj >= kMaxAdjust) sh->failed = 1u;
  // lw stays an upper bound of w's length (a leading zero limb after w -= 1
  // is harmless to every later operation)
  return lw;
}

// w ~ B^h / v (within two units) for a divisor with k1 >= 2 significant
// limbs and h >= k1, by the signed Newton steps of the header comment.
// Leaves w in bf.W and returns its limb count.
// adjust (nullable): adjust[0] += Newton steps, adjust[1] += steps taken on
// the negative branch (e <= 0).
__device__ inline int shifted_inverse(const uint32_t* v, int k1, int h, Bufs& bf, Shared* sh,
                                      char* smem, int64_t* adjust) {
  if (threadIdx.x == 0) {
    const unsigned __int128 w0 = seed_inverse(v, k1);
#pragma unroll
    for (int i = 0; i < 4; ++i) sh->w0[i] = (uint32_t)(w0 >> (32 * i));
  }
  __syncthreads();
  // w0 ~ B^(k1+2) / v; a quotient of at most two limbs (h < k1 + 2) takes
  // w0 / B^(k1+2-h) instead, within one unit of B^h / v as well
  int cur = k1 + 2;
  const int d0 = cur > h ? cur - h : 0;
  for (int i = threadIdx.x; i < 4; i += blockDim.x) bf.W[i] = i + d0 < 4 ? sh->w0[i + d0] : 0u;
  __syncthreads();
  cur -= d0;
  int lw = max(wg_prec(bf.W, 4, sh), 1);
  // the first steps on wave 0 alone (see wave_newton_early)
  if (cur < h) {
    if (wave_id() == 0) {
      int c2 = cur, l2 = lw;
      bool f = false;
      wave_newton_early(v, k1, h, bf.W, smem, adjust, c2, l2, f);
      if (lane_id() == 0) {
        sh->early_cur = c2;
        sh->early_lw = l2;
        if (f) sh->failed = 1u;
      }
    }
    __syncthreads();
    cur = sh->early_cur;
    lw = sh->early_lw;
    if (sh->failed) return lw;
  }
  // Newton steps: w ~ B^cur / v carries p = cur - k1 limbs of precision, and
  // a step to p' = p + m only needs the divisor to p' + kGuard limbs: with V
  // the top t of them (v = V B^s + low), w also approximates B^(cur-s) / V
  // to within B^(1 - kGuard) units of the same value, so each step runs on V
  // at the scale c = cur - s.  m = cur - k1 - 1 keeps one guard limb.
  while (cur < h) {
    const int m = min(h - cur, cur - k1 - 1);
    const int t = min(k1, cur + m - k1 + 1 + kGuard);
    const int sdrop = k1 - t;
    const uint32_t* V = v + sdrop;
    const int c = cur - sdrop;
    // powDiff: e = B^c - V w with |e| < 3 V < B^(t+1); since c >= t + 2,
    // (V w) mod B^(t+2) ends in limb 0 when V w >= B^c (then |e| = that
    // residue) and in an all-ones limb when V w < B^c (then e = its negation)
    const int le = t + 2;
    wg_mul(bf.E, V, t, bf.W, lw, smem, le, adjust);
    // every wave reads the same limb after the multiply's closing barrier
    const uint32_t top = __builtin_amdgcn_readfirstlane(bf.E[le - 1]);
    const bool neg = top == 0u;
    if (!neg) {
      if (top != 0xffffffffu) {   // outside the error bound: never expected
        if (threadIdx.x == 0) sh->failed = 1u;
        __syncthreads();
        break;
      }
      auto X = [&](int) -> uint32_t { return 0u; };
      auto Y = [&](int j) -> uint32_t { return bf.E[j]; };
      div_addsub<true>(bf.E, le, X, Y, sh);   // e = 0 - (V w mod B^le), in place
    }
    if (adjust) {
      adjust[0] += 1;
      adjust[1] += neg ? 1 : 0;
    }
    // step: Y = w |e|, of which floor(Y / B^(c-m)) is needed; the low sd
    // limbs of |e| add less than w B^sd <= B^(c-m-1) to Y, so dropping them
    // moves that quotient by at most one unit (inside the error bound)
    const int sd = max(0, min(le - 1, c - m - 1 - lw));
    const int sy = c - m - sd;           // Y / B^sy
    // only the limbs from sy up are needed: a high product, which may come
    // out one unit low (inside the error bound as well)
    const bool exact = wg_mul(bf.T, bf.W, lw, bf.E + sd, le - sd, smem, -1, adjust, sy);
    const int ly = lw + le - sd;
    // negative branch: the ceiling takes one more unit unless the dropped
    // limbs Y[0 .. sy) are all zero (nullUpToInd); when the high product left
    // them out it always takes it (one unit more at most)
    uint32_t cin = 0u;
    if (neg) {
      if (exact) {
        int nz = 0;
        for (int j = threadIdx.x; j < min(sy, ly); j += blockDim.x) nz |= bf.T[j] != 0u;
        cin = __syncthreads_or(nz) ? 1u : 0u;
      } else {
        cin = 1u;
      }
    }
    const int lnew = lw + m + 1;
    auto X = [&](int j) -> uint32_t { return (j >= m && j - m < lw) ? bf.W[j - m] : 0u; };
    auto Y = [&](int j) -> uint32_t { return j + sy < ly ? bf.T[j + sy] : 0u; };
    // (the reset happens before every thread's atomicMax: the addition's
    // carry scan synchronises the work-group first)
    if (threadIdx.x == 0) sh->red[3] = 0;
    if (neg) div_addsub<true>(bf.U2, lnew, X, Y, sh, &sh->red[3], cin);
    else div_addsub<false>(bf.U2, lnew, X, Y, sh, &sh->red[3]);
    {  // the new w is in U2: swap the two buffers instead of copying
      uint32_t* tmp = bf.W;
      bf.W = bf.U2;
      bf.U2 = tmp;
    }
    lw = max((int)sh->red[3], 1);   // w's length, from the addition itself
    __syncthreads();
    cur += m;
  }
  return lw;
}

// q[0..nq), r[0..nr) = divmod(u[0..nu), v[0..nv)); returns the status.
// With inverse_only, writes floor(B^h_inv / v) into q[0..nq) instead.
// adjust (nullable, 3 ints): Newton steps, fix-up unit steps, quotient
// corrections, each added to.
__device__ inline int wg_divmod(uint32_t* q, int nq, uint32_t* r, int nr, const uint32_t* u, int nu,
                                const uint32_t* v, int nv, Bufs bf, Shared* sh, char* smem,
                                bool inverse_only, int h_inv, int64_t* adjust) {
  if (threadIdx.x == 0) sh->failed = 0u;
  __syncthreads();
  int k1, hu;
  if (inverse_only) {
    k1 = wg_prec(v, nv, sh);
    hu = h_inv;
  } else {
    wg_prec2(v, nv, u, nu, sh, &k1, &hu);
  }
  if (k1 == 0) {
    if (!inverse_only) {
      wg_fill(q, nq, 0u);
      wg_shr_copy(r, nr, u, nu, 0);
    } else {
      wg_fill(q, nq, 0u);
    }
    return BIGINT_DIVZERO;
  }
  const int h = hu;
  if (!inverse_only && h < k1) {  // u < v
    wg_fill(q, nq, 0u);
    wg_shr_copy(r, nr, u, nu, 0);
    return BIGINT_DIV_OK;
  }
  if (k1 == 1) {
    // short division by one limb (one lane walks the limbs top down)
    const uint32_t d = v[0];
    if (!inverse_only) wg_fill(q, nq, 0u);
    else wg_fill(q, nq, 0u);
    if (threadIdx.x == 0) {
      uint64_t rem = 0;
      for (int i = h - (inverse_only ? 0 : 1); i >= 0; --i) {
        const uint32_t limb = inverse_only ? (i == h ? 1u : 0u) : u[i];
        const uint64_t t = (rem << 32) | limb;
        const uint64_t qq = t / d;
        rem = t - qq * d;
        if (i < nq) q[i] = (uint32_t)qq;
      }
      if (!inverse_only) {
        for (int i = 0; i < nr; ++i) r[i] = i == 0 ? (uint32_t)rem : 0u;
      }
    }
    __syncthreads();
    return BIGINT_DIV_OK;
  }
  int lw = shifted_inverse(v, k1, h, bf, sh, smem, adjust);
  if (inverse_only) {
    // the diagnostic wants floor(B^h / v) exactly: one exact fix-up at scale h
    lw = fixup(v, k1, h, bf, lw, sh, smem, nullptr);
    wg_shr_copy(q, nq, bf.W, lw, 0);
    return sh->failed ? BIGINT_DIV_FAILED : BIGINT_DIV_OK;
  }
  // q~ = floor(u w / B^h), from the top limbs of u only: the low su limbs add
  // less than B^(su+lw) <= B^(h-1) to u w, so they move q~ by at most one
  // unit; a high product (limbs from h - su up) takes at most one more
  const int su = max(0, h - 1 - lw);
  wg_mul(bf.T, u + su, h - su, bf.W, lw, smem, -1, adjust, h - su);
  const uint32_t* qt = bf.T + (h - su);              // q~: lw limbs
  const int lq = max(wg_prec(qt, lw, sh), 1);
  // r~ = u - q~ v; |r~| < 8 v < B^(k1+1), so r~ mod B^(k1+2) holds it with
  // its sign in the top limb
  const int lr = k1 + 2;
  wg_mul(bf.U2, qt, lq, v, k1, smem, lr, adjust);
  wg_arith<true>(bf.E, lr, u, h, bf.U2, min(lr, lq + k1), sh);
  // corrections: while r~ < 0, r~ += v (q~ - 1); while r~ >= v, r~ -= v (q~ + 1)
  // (each loop is bounded; leaving one at its bound marks the division failed,
  // which the error analysis rules out: at most 4 corrections are possible)
  int dq = 0;
  bool done_neg = false, done_pos = false;
  for (int rounds = 0; rounds < 8; ++rounds) {
    const uint32_t top = __builtin_amdgcn_readfirstlane(bf.E[lr - 1]);
    if (top == 0u) { done_neg = true; break; }
    wg_arith<false>(bf.E, lr, bf.E, lr, v, k1, sh);
    --dq;
  }
  for (int rounds = 0; rounds < 8 && done_neg; ++rounds) {
    if (wg_cmp(bf.E, lr, v, k1, lr, sh) < 0) { done_pos = true; break; }
    wg_arith<true>(bf.E, lr, bf.E, lr, v, k1, sh);
    ++dq;
  }
  if (!done_pos && threadIdx.x == 0) sh->failed = 1u;
  if (adjust) adjust[2] += dq < 0 ? -dq : dq;
  // q = q~ + dq over all nq limbs and r = r~ over nr limbs, in one pass
  // (r's copy rides along with the addition's first round)
  for (int i = threadIdx.x; i < nr; i += blockDim.x) r[i] = i < k1 ? bf.E[i] : 0u;
  if (dq >= 0) wg_arith1<false>(q, nq, qt, lq, (uint32_t)dq, sh);
  else wg_arith1<true>(q, nq, qt, lq, (uint32_t)(-dq), sh);
  return sh->failed ? BIGINT_DIV_FAILED : BIGINT_DIV_OK;
}

}  // namespace div
}  // namespace bi
