// dev_mul_plain.hpp -- the plain multiply of Section 5.2 on u64 digits.
//
// The product digits C_k = sum_{i+j=k} A_i B_j (Section 5.2) are computed in
// blocks of Q consecutive outputs.  A block is evaluated like halfConv: one
// loop over the index range common to all Q outputs, whose inner loop of
// count Q reuses a sliding window of Q digits of B held in registers, plus
// the two small triangles that only some outputs need.  Every partial sum is
// a (low, high, carry) triple of u64 (oneConvMul), and combineQ folds the Q
// triples into Q digits plus two spill digits.  The low digits of all blocks
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

// acc += x * y (64 x 64 -> 128 bits, plus an overflow count)
__device__ __forceinline__ void mac64(Acc3& a, uint64_t x, uint64_t y) {
  const uint64_t plo = x * y;
  const uint64_t phi = __umul64hi(x, y);
  unsigned long long c1, c2;
  a.lo = __builtin_addcll(a.lo, plo, 0ull, &c1);
  a.hi = __builtin_addcll(a.hi, phi, c1, &c2);
  a.cc += c2;
}

__device__ __forceinline__ void add_into(uint64_t& tl, uint64_t& th, uint64_t v) {
  unsigned long long c;
  tl = __builtin_addcll(tl, v, 0ull, &c);
  th += c;
}

// LDS bytes needed by wg_mul_plain for an (na x nb)-limb product
__host__ __device__ inline size_t plain_lds_bytes(int na, int nb) {
  const int ma = (na + 1) / 2, mb = (nb + 1) / 2;
  return (size_t)(ma + mb) * 8 + 64;
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

  // stage the operands as u64 digits (two u32 limbs each, odd count padded)
  for (int i = t; i < ma; i += T) {
    const uint64_t lo = a[2 * i], hi = (2 * i + 1 < na) ? a[2 * i + 1] : 0u;
    A[i] = lo | (hi << 32);
  }
  for (int i = t; i < mb; i += T) {
    const uint64_t lo = b[2 * i], hi = (2 * i + 1 < nb) ? b[2 * i + 1] : 0u;
    Bd[i] = lo | (hi << 32);
  }
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
    Acc3 acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = Acc3{0, 0, 0};

    // index range common to all Q outputs
    const int I_lo = max(0, k0 + Q - mb);
    const int I_hi = min(k0, ma - 1);
    const bool common = I_lo <= I_hi;
    if (common) {
      // window w[q] = B[k0 - i + q], walking i downwards from I_hi
      uint64_t w[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) w[q] = Bd[k0 - I_hi + q];
      for (int i = I_hi; i >= I_lo; --i) {
        const uint64_t x = A[i];
#pragma unroll
        for (int q = 0; q < Q; ++q) mac64(acc[q], x, w[q]);
        if (i > I_lo) {
#pragma unroll
          for (int q = 0; q < Q - 1; ++q) w[q] = w[q + 1];
          w[Q - 1] = Bd[k0 - i + Q];
        }
      }
    }
    // the triangles (or the whole range when nothing is common)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int k = k0 + q;
      const int lo = max(0, k - mb + 1), hi = min(k, ma - 1);
      if (!common) {
        for (int i = lo; i <= hi; ++i) mac64(acc[q], A[i], Bd[k - i]);
      } else {
        for (int i = lo; i < I_lo; ++i) mac64(acc[q], A[i], Bd[k - i]);
        for (int i = I_hi + 1; i <= hi; ++i) mac64(acc[q], A[i], Bd[k - i]);
      }
    }
    // combineQ: Q triples -> Q digits + 2 spill digits
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
        sp0[r] = d;
      } else {
        sp1[r] = d;
      }
    }
  }
  __syncthreads();  // operands dead: reuse their LDS for the spills

  uint64_t* Sp = sm;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int blk = (r & 1) ? (r + 1) * T - 1 - t : r * T + t;
    if (blk < NBLK) { Sp[2 * blk] = sp0[r]; Sp[2 * blk + 1] = sp1[r]; }
  }
  __syncthreads();

  // out += spills: block blk's two spill digits sit at digit (blk+1)Q + e
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

}  // namespace bi
