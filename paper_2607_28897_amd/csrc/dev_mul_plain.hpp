// dev_mul_plain.hpp -- the plain multiply of Section 5.2 on u64 digits.
//
// The product digits C_k = sum_{i+j=k} A_i B_j (Section 5.2) are computed in
// blocks of Q consecutive outputs.  A block is evaluated like halfConv: one
// loop over the index range common to all Q outputs, whose inner loop of
// count Q reuses a sliding window of Q digits of B held in registers, plus
// the two small triangles that only some outputs need.  Every partial sum is
// kept as column sums of 32 x 32-bit products with carry counts (AccCol) and
// folded at the end into the (low, high, carry) triple of u64 that
// oneConvMul keeps; combineQ folds the Q triples into Q digits plus two spill
// digits.  The low digits of all blocks
// tile the product; the spills, shifted by Q, are added to them with one
// work-group carry scan -- the Lsh + Hsh addition of bmulReg.
//
// Balance: output k of an m x m product costs min(k+1, 2m-1-k) digit
// products.  Thread t takes blocks t, 2T-1-t, 2T+t, 4T-1-t (threadConv's
// forward/mirrored pairing applied to the rising and to the falling half of
// the full product), so with 4T blocks every thread does the same work.
#pragma once

#include "common.hpp"
#include "dev_addsub.hpp"

namespace bi {

struct Acc3 {
  uint64_t lo, hi, cc;
};

// Sum of 64 x 64 -> 128-bit digit products, kept as column sums of 32 x
// 32-bit products: value = s0 + s1 2^32 + s2 2^64 + c0 2^64 + c1 2^96 +
// c2 2^128, where c0..c2 count the carries out of bit 63 of s0..s2.  One
// digit product is four v_mad_u64_u32 (32 x 32 + 64 bits, carry out to a
// lane mask; x0 y1 and x1 y0 both go to s1) and four carry additions.
struct AccCol {
  uint64_t s0, s1, s2;  // column sums at bits 0, 32, 64
  uint32_t c0, c1, c2;  // carries out of bit 63 of each
};

__device__ __forceinline__ void acc_zero(AccCol& a) {
  a.s0 = a.s1 = a.s2 = 0;
  a.c0 = a.c1 = a.c2 = 0;
}

// a += x * y.  The four multiply-adds go first and the carry additions after
// them, so every carry mask is read three or more instructions after it is
// written.
__device__ __forceinline__ void mac64(AccCol& a, uint64_t x, uint64_t y) {
  const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
  const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32);
  uint64_t k0, k1, k2, k3;
  asm("v_mad_u64_u32 %0, %6, %10, %12, %0\n\t"
      "v_mad_u64_u32 %1, %7, %10, %13, %1\n\t"
      "v_mad_u64_u32 %2, %8, %11, %13, %2\n\t"
      "v_mad_u64_u32 %1, %9, %11, %12, %1\n\t"
      "v_addc_co_u32_e64 %3, %6, 0, %3, %6\n\t"
      "v_addc_co_u32_e64 %4, %7, 0, %4, %7\n\t"
      "v_addc_co_u32_e64 %5, %8, 0, %5, %8\n\t"
      "v_addc_co_u32_e64 %4, %9, 0, %4, %9"
      : "+v"(a.s0), "+v"(a.s1), "+v"(a.s2), "+v"(a.c0), "+v"(a.c1), "+v"(a.c2),
        "=&s"(k0), "=&s"(k1), "=&s"(k2), "=&s"(k3)
      : "v"(x0), "v"(x1), "v"(y0), "v"(y1));
}

// a += x * ya and b += x * yb in one block: the compiler separates inline asm
// blocks with a wait state (it cannot see which carry masks they share), so
// fewer, longer blocks issue faster.  Carry masks are read four or more
// instructions after they are written.
__device__ __forceinline__ void mac64x2(AccCol& a, AccCol& b, uint64_t x, uint64_t ya, uint64_t yb) {
  const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
  const uint32_t a0 = (uint32_t)ya, a1 = (uint32_t)(ya >> 32);
  const uint32_t b0 = (uint32_t)yb, b1 = (uint32_t)(yb >> 32);
  uint64_t k0, k1, k2, k3, k4, k5, k6, k7;
  asm("v_mad_u64_u32 %0, %12, %20, %22, %0\n\t"
      "v_mad_u64_u32 %1, %13, %20, %23, %1\n\t"
      "v_mad_u64_u32 %2, %14, %21, %23, %2\n\t"
      "v_mad_u64_u32 %1, %15, %21, %22, %1\n\t"
      "v_mad_u64_u32 %6, %16, %20, %24, %6\n\t"
      "v_mad_u64_u32 %7, %17, %20, %25, %7\n\t"
      "v_mad_u64_u32 %8, %18, %21, %25, %8\n\t"
      "v_mad_u64_u32 %7, %19, %21, %24, %7\n\t"
      "v_addc_co_u32_e64 %3, %12, 0, %3, %12\n\t"
      "v_addc_co_u32_e64 %4, %13, 0, %4, %13\n\t"
      "v_addc_co_u32_e64 %5, %14, 0, %5, %14\n\t"
      "v_addc_co_u32_e64 %4, %15, 0, %4, %15\n\t"
      "v_addc_co_u32_e64 %9, %16, 0, %9, %16\n\t"
      "v_addc_co_u32_e64 %10, %17, 0, %10, %17\n\t"
      "v_addc_co_u32_e64 %11, %18, 0, %11, %18\n\t"
      "v_addc_co_u32_e64 %10, %19, 0, %10, %19"
      : "+v"(a.s0), "+v"(a.s1), "+v"(a.s2), "+v"(a.c0), "+v"(a.c1), "+v"(a.c2),
        "+v"(b.s0), "+v"(b.s1), "+v"(b.s2), "+v"(b.c0), "+v"(b.c1), "+v"(b.c2),
        "=&s"(k0), "=&s"(k1), "=&s"(k2), "=&s"(k3), "=&s"(k4), "=&s"(k5), "=&s"(k6), "=&s"(k7)
      : "v"(x0), "v"(x1), "v"(a0), "v"(a1), "v"(b0), "v"(b1));
}

// the (lo, hi, carry) triple of 64-bit digits that an AccCol stands for
__device__ __forceinline__ Acc3 acc_fold(const AccCol& a) {
  // value = s0 + s1 2^32 + (s2 + c0) 2^64 + c1 2^96 + c2 2^128
  unsigned long long k1, k2, k3, k4;
  Acc3 r;
  r.lo = __builtin_addcll(a.s0, a.s1 << 32, 0ull, &k1);
  uint64_t hi = __builtin_addcll(a.s2, (a.s1 >> 32) + k1, 0ull, &k2);  // (s1>>32)+k1 < 2^32+1
  hi = __builtin_addcll(hi, (uint64_t)a.c0, 0ull, &k3);
  hi = __builtin_addcll(hi, (uint64_t)a.c1 << 32, 0ull, &k4);
  r.hi = hi;
  r.cc = (uint64_t)a.c2 + k2 + k3 + k4;
  return r;
}

__device__ __forceinline__ void add_into(uint64_t& tl, uint64_t& th, uint64_t v) {
  unsigned long long c;
  tl = __builtin_addcll(tl, v, 0ull, &c);
  th += c;
}

// LDS bytes needed by wg_mul_plain for an (na x nb)-limb product: the two
// operands as u64 digits, then 64 bytes of carry-scan scratch (whose first
// digit the common loop may read, unused, just past B)
__host__ __device__ inline size_t plain_lds_bytes(int na, int nb) {
  const int ma = (na + 1) / 2, mb = (nb + 1) / 2;
  return (size_t)(ma + mb) * 8 + 64;
}

// Column sums of the Q outputs of the block starting at digit k0 over the
// index range i in [lo, hi] of A (every output of the block has all those
// terms): one loop whose inner loop of count Q reuses a sliding window of Q
// digits of B held in registers.
template <int Q>
__device__ __forceinline__ void plain_common(AccCol (&col)[Q], const uint64_t* A, const uint64_t* Bd,
                                             int k0, int lo, int hi, int mb) {
  // window w[q] = B[k0 - i + q], walking i downwards from hi
  uint64_t w[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) w[q] = Bd[k0 - hi + q];
  int i = hi;
  // rounds of Q steps.  Step j of a round (from i) has the window
  // B[k0 - i + j + q] = w[q + j], or nx[q + j - Q] past the ring's end,
  // so the ring turns at compile time and the round's digits of A and
  // of B are read at its start.  A round reads B up to index
  // k0 - i + 2Q - 1 <= k0 - lo + Q <= mb (lo is at least the block's common
  // lower bound k0 + Q - mb): at most one digit past B, the first of the
  // scratch area that follows it in LDS (always allocated); that value is
  // never used.  Unclamped, the Q reads share one address.
  static_assert(Q % 2 == 0, "columns go in pairs");
  // one round from i with window `win`; the round's new digits go to `nw`
  auto round = [&](int i0, const uint64_t (&win)[Q], uint64_t (&nw)[Q]) {
    uint64_t x[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) x[j] = A[i0 - j];
#pragma unroll
    for (int j = 0; j < Q; ++j) nw[j] = Bd[k0 - i0 + Q + j];
#pragma unroll
    for (int j = 0; j < Q; ++j)
#pragma unroll
      for (int q = 0; q < Q; q += 2)
        mac64x2(col[q], col[q + 1], x[j], q + j < Q ? win[q + j] : nw[q + j - Q],
                q + 1 + j < Q ? win[q + 1 + j] : nw[q + 1 + j - Q]);
  };
  // two rounds per pass, the rings swapping roles (no register moves)
  uint64_t v[Q];
  for (; i - (2 * Q - 1) >= lo; i -= 2 * Q) {
    round(i, w, v);
    round(i - Q, v, w);
  }
  if (i - (Q - 1) >= lo) {
    round(i, w, v);
#pragma unroll
    for (int q = 0; q < Q; ++q) w[q] = v[q];
    i -= Q;
  }
  // the last steps one at a time
  for (; i >= lo; --i) {
    const uint64_t x = A[i];
    // the window's next digit, read before it is needed (clamped: the
    // value read after the last step is not used)
    const uint64_t nxt = Bd[min(k0 - i + Q, mb - 1)];
#pragma unroll
    for (int q = 0; q < Q; ++q) mac64(col[q], x, w[q]);
#pragma unroll
    for (int q = 0; q < Q - 1; ++q) w[q] = w[q + 1];
    w[Q - 1] = nxt;
  }
}

// The terms of the block's outputs outside the common range [I_lo, I_hi]
// (the two triangles), or all of them when nothing is common.
template <int Q>
__device__ __forceinline__ void plain_triangles(AccCol (&col)[Q], const uint64_t* A, const uint64_t* Bd,
                                                int k0, int ma, int mb, int I_lo, int I_hi, bool common) {
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k = k0 + q;
    const int lo = max(0, k - mb + 1), hi = min(k, ma - 1);
    if (!common) {
      for (int i = lo; i <= hi; ++i) mac64(col[q], A[i], Bd[k - i]);
    } else {
      for (int i = lo; i < I_lo; ++i) mac64(col[q], A[i], Bd[k - i]);
      for (int i = I_hi + 1; i <= hi; ++i) mac64(col[q], A[i], Bd[k - i]);
    }
  }
}

// combineQ: the block's Q triples -> Q output digits (stored) + 2 spill digits
template <int Q>
__device__ __forceinline__ void plain_block_out(const Acc3 (&acc)[Q], uint32_t* out, int nout, int k0,
                                                uint64_t& sp0, uint64_t& sp1) {
  uint64_t tl = 0, th = 0;
#pragma unroll
  for (int j = 0; j < Q + 2; ++j) {
    if (j < Q) add_into(tl, th, acc[j].lo);
    if (j >= 1 && j <= Q) add_into(tl, th, acc[j - 1].hi);
    if (j >= 2) add_into(tl, th, acc[j - 2].cc);
    const uint64_t d = tl;
    tl = th; th = 0;
    if (j < Q) {
      const int l = 2 * (k0 + j);
      if (l < nout) out[l] = (uint32_t)d;
      if (l + 1 < nout) out[l + 1] = (uint32_t)(d >> 32);
    } else if (j == Q) {
      sp0 = d;
    } else {
      sp1 = d;
    }
  }
}

// out += the spills: block blk's two spill digits sit at digit (blk+1)Q + e;
// one work-group carry scan (the Lsh + Hsh addition of bmulReg)
template <int Q>
__device__ __forceinline__ void plain_add_spills(uint32_t* out, int nout, const uint64_t* Sp,
                                                 uint32_t* scratch) {
  auto X = [&](int j) -> uint32_t { return out[j]; };
  auto Y = [&](int j) -> uint32_t {
    const int pd = j >> 1;
    if (pd < Q) return 0u;
    const int e = pd % Q;
    if (e >= 2) return 0u;
    const uint64_t d = Sp[2 * (pd / Q - 1) + e];
    return (j & 1) ? (uint32_t)(d >> 32) : (uint32_t)d;
  };
  wg_addsub<8, false, decltype(X), decltype(Y), true>(out, nout, X, Y, 0u, scratch);
}

// stage the operands as u64 digits (two u32 limbs each, odd count padded)
__device__ __forceinline__ void plain_stage(uint64_t* A, uint64_t* Bd, const uint32_t* __restrict__ a,
                                            int na, const uint32_t* __restrict__ b, int nb) {
  const int ma = (na + 1) / 2, mb = (nb + 1) / 2;
  for (int i = threadIdx.x; i < ma; i += blockDim.x) {
    const uint64_t lo = a[2 * i], hi = (2 * i + 1 < na) ? a[2 * i + 1] : 0u;
    A[i] = lo | (hi << 32);
  }
  for (int i = threadIdx.x; i < mb; i += blockDim.x) {
    const uint64_t lo = b[2 * i], hi = (2 * i + 1 < nb) ? b[2 * i + 1] : 0u;
    Bd[i] = lo | (hi << 32);
  }
}

// out[0 .. na+nb) = a[0..na) * b[0..nb); one work-group, R blocks of Q
// output digits per thread (R*blockDim*Q >= ma+mb required).
template <int Q, int R>
__device__ __forceinline__ void wg_mul_plain(uint32_t* out, const uint32_t* __restrict__ a, int na,
                             const uint32_t* __restrict__ b, int nb, uint64_t* sm) {
  const int ma = (na + 1) / 2, mb = (nb + 1) / 2;
  const int nout = na + nb;
  uint64_t* A = sm;
  uint64_t* Bd = sm + ma;
  uint32_t* scratch = reinterpret_cast<uint32_t*>(sm + ma + mb);
  const int T = blockDim.x, t = threadIdx.x;

  plain_stage(A, Bd, a, na, b, nb);
  __syncthreads();

  const int K = ma + mb;
  const int NBLK = (K + Q - 1) / Q;
  uint64_t sp0[R], sp1[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int blk = (r & 1) ? (r + 1) * T - 1 - t : r * T + t;
    sp0[r] = 0; sp1[r] = 0;
    if (blk >= NBLK) continue;
    const int k0 = blk * Q;
    AccCol col[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc_zero(col[q]);
    // index range common to all Q outputs
    const int I_lo = max(0, k0 + Q - mb);
    const int I_hi = min(k0, ma - 1);
    const bool common = I_lo <= I_hi;
    if (common) plain_common<Q>(col, A, Bd, k0, I_lo, I_hi, mb);
    plain_triangles<Q>(col, A, Bd, k0, ma, mb, I_lo, I_hi, common);
    Acc3 acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = acc_fold(col[q]);
    plain_block_out<Q>(acc, out, nout, k0, sp0[r], sp1[r]);
  }
  __syncthreads();  // operands dead: reuse their LDS for the spills

  uint64_t* Sp = sm;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int blk = (r & 1) ? (r + 1) * T - 1 - t : r * T + t;
    if (blk < NBLK) { Sp[2 * blk] = sp0[r]; Sp[2 * blk + 1] = sp1[r]; }
  }
  __syncthreads();
  plain_add_spills<Q>(out, nout, Sp, scratch);
}

// LDS bytes of wg_mul_plain_split: wg_mul_plain's, then the partial column
// sums of parts 1..S-1 (threads per part Tp, Q triples each)
__host__ __device__ inline size_t plain_split_lds_bytes(int na, int nb, int S, int Tp, int Q) {
  return plain_lds_bytes(na, nb) + (size_t)(S - 1) * Tp * Q * sizeof(Acc3);
}

// wg_mul_plain with every block's common index range cut into S parts, for
// batches too small to give every SIMD waves of its own: thread
// (s, t) = (threadIdx.x / Tp, threadIdx.x % Tp), Tp = blockDim.x / S, sums
// part s of the blocks thread t has in wg_mul_plain (part 0 also takes the
// triangles), and part 0 adds the other parts' (lo, hi, carry) triples from
// LDS before combineQ.  The digits computed are those of wg_mul_plain.
template <int Q, int R, int S>
__device__ __forceinline__ void wg_mul_plain_split(uint32_t* out, const uint32_t* __restrict__ a, int na,
                                                   const uint32_t* __restrict__ b, int nb, uint64_t* sm) {
  static_assert(S >= 2, "one part is wg_mul_plain");
  const int ma = (na + 1) / 2, mb = (nb + 1) / 2;
  const int nout = na + nb;
  uint64_t* A = sm;
  uint64_t* Bd = sm + ma;
  uint32_t* scratch = reinterpret_cast<uint32_t*>(sm + ma + mb);
  Acc3* part = reinterpret_cast<Acc3*>(sm + ma + mb + 8);  // past the 64-byte scratch
  const int Tp = blockDim.x / S, t = threadIdx.x % Tp, s = threadIdx.x / Tp;

  plain_stage(A, Bd, a, na, b, nb);
  __syncthreads();

  const int K = ma + mb;
  const int NBLK = (K + Q - 1) / Q;
  uint64_t sp0[R], sp1[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int blk = (r & 1) ? (r + 1) * Tp - 1 - t : r * Tp + t;
    sp0[r] = 0; sp1[r] = 0;
    const bool live = blk < NBLK;
    const int k0 = blk * Q;
    AccCol col[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc_zero(col[q]);
    if (live) {
      const int I_lo = max(0, k0 + Q - mb);
      const int I_hi = min(k0, ma - 1);
      const bool common = I_lo <= I_hi;
      if (common) {
        // part s: indices [hi_s - len + 1, hi_s] of the common range, from the top
        const int len = (I_hi - I_lo + S) / S;
        const int hi_s = I_hi - s * len;
        const int lo_s = max(I_lo, hi_s - len + 1);
        if (lo_s <= hi_s) plain_common<Q>(col, A, Bd, k0, lo_s, hi_s, mb);
      }
      if (s == 0) plain_triangles<Q>(col, A, Bd, k0, ma, mb, I_lo, I_hi, common);
    }
    Acc3 acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = acc_fold(col[q]);
    if (s > 0) {
#pragma unroll
      for (int q = 0; q < Q; ++q) part[((s - 1) * Tp + t) * Q + q] = acc[q];
    }
    __syncthreads();
    if (s == 0 && live) {
      for (int p = 1; p < S; ++p) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const Acc3 o = part[((p - 1) * Tp + t) * Q + q];
          unsigned long long c1, c2;
          acc[q].lo = __builtin_addcll(acc[q].lo, o.lo, 0ull, &c1);
          acc[q].hi = __builtin_addcll(acc[q].hi, o.hi, c1, &c2);
          acc[q].cc += o.cc + c2;
        }
      }
      plain_block_out<Q>(acc, out, nout, k0, sp0[r], sp1[r]);
    }
    __syncthreads();  // the partials are rewritten by the next block
  }

  uint64_t* Sp = sm;  // operands dead: their LDS takes the spills
  if (s == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int blk = (r & 1) ? (r + 1) * Tp - 1 - t : r * Tp + t;
      if (blk < NBLK) { Sp[2 * blk] = sp0[r]; Sp[2 * blk + 1] = sp1[r]; }
    }
  }
  __syncthreads();
  plain_add_spills<Q>(out, nout, Sp, scratch);
}

}  // namespace bi
