// kernels_kara.hip -- one Karatsuba level over the MFMA-split multiply.
//
// With h = ceil(n/2), a = a1 B^h + a0 and b = b1 B^h + b0 (a0, b0: h limbs;
// a1, b1: n - h limbs):
//   a b = p2 B^(2h) + (p0 + p2 + s pm) B^h + p0,
//   p0 = a0 b0, p2 = a1 b1, pm = |a0 - a1| |b1 - b0|,
//   s = sign(a0 - a1) sign(b1 - b0),
// since a0 b1 + a1 b0 = (a0 - a1)(b1 - b0) + a0 b0 + a1 b1.  Three products
// of half the size replace one: 3/4 of the multiply-accumulates, for one
// linear pass before (both differences) and one after.
#include "internal.hpp"
#include "dev_addsub.hpp"
#include "dev_mul_mfma.hpp"

namespace bi {

// d = |x - y| over n limbs and sgn = sign(x - y) (x: nx limbs, y: ny limbs,
// zero-extended; n <= 16 * blockDim.x).  Both differences are formed in the
// same pass; the borrow out of x - y picks one.  blockIdx.y = 0: x = a0,
// y = a1; = 1: x = b1, y = b0.  VEC: every run of four limbs is read and
// written with one 16-byte access (n a multiple of 8, so h, nx and ny are
// multiples of 4, and the buffers 16-byte aligned).
constexpr int kKaraQ = 16;

template <bool VEC>
__global__ __launch_bounds__(1024) void k_kara_diff(uint32_t* ws, int64_t ws_stride, int32_t* sgn,
                                                    const uint32_t* a, const uint32_t* b, int n,
                                                    int h) {
  __shared__ uint32_t scratch[32];
  const int64_t inst = blockIdx.x;
  const bool side_b = blockIdx.y == 1;
  const uint32_t* base = (side_b ? b : a) + inst * n;
  const uint32_t* lo = base;
  const uint32_t* hi = base + h;
  const uint32_t* x = side_b ? hi : lo;
  const uint32_t* y = side_b ? lo : hi;
  const int nx = side_b ? n - h : h, ny = side_b ? h : n - h;
  uint32_t* d = ws + inst * ws_stride + (side_b ? h : 0);
  const int j0 = threadIdx.x * kKaraQ;
  const int valid = min(kKaraQ, max(0, h - j0));
  uint32_t xv[kKaraQ], yv[kKaraQ];
  if (VEC) {
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int i = 0; i < kKaraQ; i += 4) {
      const int j = j0 + i;
      const uint4 xa = (i < valid && j < nx) ? *reinterpret_cast<const uint4*>(x + j) : z;
      const uint4 ya = (i < valid && j < ny) ? *reinterpret_cast<const uint4*>(y + j) : z;
      xv[i] = xa.x; xv[i + 1] = xa.y; xv[i + 2] = xa.z; xv[i + 3] = xa.w;
      yv[i] = ya.x; yv[i + 1] = ya.y; yv[i + 2] = ya.z; yv[i + 3] = ya.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kKaraQ; ++i) {
      const int j = j0 + i;
      const uint32_t xa = x[max(min(j, nx - 1), 0)], ya = y[max(min(j, ny - 1), 0)];
      xv[i] = (i < valid && j < nx) ? xa : 0u;
      yv[i] = (i < valid && j < ny) ? ya : 0u;
    }
  }
  LimbRun<kKaraQ, true> r1, r2;
  r1.build(xv, yv, valid);
  r2.build(yv, xv, valid);
  uint32_t borrow;
  const uint32_t c1 = wg_carry_scan(r1.G, r1.P, 0u, scratch, &borrow);
  r1.apply(c1);
  uint32_t unused;
  const uint32_t c2 = wg_carry_scan(r2.G, r2.P, 0u, scratch, &unused);
  r2.apply(c2);
  bool nz = false;
#pragma unroll
  for (int i = 0; i < kKaraQ; ++i) nz |= r1.s[i] != 0u;
  const bool any = __syncthreads_or(nz);
  if (VEC) {
#pragma unroll
    for (int i = 0; i < kKaraQ; i += 4)
      if (i < valid)
        *reinterpret_cast<uint4*>(d + j0 + i) =
            borrow ? make_uint4(r2.s[i], r2.s[i + 1], r2.s[i + 2], r2.s[i + 3])
                   : make_uint4(r1.s[i], r1.s[i + 1], r1.s[i + 2], r1.s[i + 3]);
  } else {
#pragma unroll
    for (int i = 0; i < kKaraQ; ++i)
      if (i < valid) d[j0 + i] = borrow ? r2.s[i] : r1.s[i];
  }
  if (threadIdx.x == 0) sgn[2 * inst + (side_b ? 1 : 0)] = borrow ? -1 : (any ? 1 : 0);
}

// The three products of every instance in one launch (blockIdx.y = job).
struct KaraJob {
  uint32_t* out;
  int64_t out_stride;
  const uint32_t* a;
  int64_t a_stride;
  const uint32_t* b;
  int64_t b_stride;
  int na, nb;
};
struct KaraJobs {
  KaraJob j[3];
};

template <int DW, int P>
__global__ __launch_bounds__(512) void k_kara_mul(KaraJobs jobs) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int64_t inst = blockIdx.x;
  const KaraJob& J = jobs.j[blockIdx.y];
  mfma::wg_mul_mfma<DW, P>(J.out + inst * J.out_stride, nullptr, J.a + inst * J.a_stride, J.na,
                           J.b + inst * J.b_stride, J.nb, smem, J.na + J.nb);
}

// out (2n limbs) = p0 + p2 B^(2h) + (p0 + p2 + s pm) B^h.  With s < 0 the
// subtraction of pm B^h becomes additions modulo B^(2n):
// -pm B^h = ~pm B^h + B^h - B^(3h), where ~pm complements the 2h limbs of pm
// and -B^(3h) is the all-ones limbs [3h, 2n).  Limb k then sums at most six
// non-negative 32-bit terms and a 1: t_k = L_k + 2^32 H_k with H_k <= 5, and
// out = sum L_k B^k + sum H_k B^(k+1) mod B^(2n), an addition whose limbs
// carry at most one.  (3h <= 2n for every n >= 2.)
//
// The output is cut into chunks of kCombChunk limbs, one work-group each, so
// that the pass runs on the whole chip: every chunk adds with carry-in 0 and
// records its carry out and whether it came out all ones; k_kara_carry then
// walks the chunks of an instance and ripples each incoming carry through the
// chunk's leading all-ones limbs.
constexpr int kCombQ = 4;
constexpr int kCombChunk = 1024 * kCombQ;
constexpr int kCombMaxChunks = 16;   // 2n <= 16 * 4096 limbs (h <= 16384)

//
// VEC (n a multiple of 8, buffers 16-byte aligned): the region bounds h, 2h,
// 3h and h + 2(n - h) are multiples of 4, so each thread's four limbs share
// one case and every source is read with one 16-byte load per run; the high
// part of the sum just below a thread's run comes from the lane below (the
// first lane of a wave evaluates it on its own).
template <bool VEC>
__global__ __launch_bounds__(1024) void k_kara_combine(uint32_t* out, const uint32_t* ws,
                                                       int64_t ws_stride, const int32_t* sgn,
                                                       uint32_t* summ, int n, int h) {
  __shared__ uint32_t scratch[32];
  const int64_t inst = blockIdx.x;
  const int chunk = blockIdx.y;
  const int k0 = chunk * kCombChunk;
  const int len = min(kCombChunk, 2 * n - k0);
  if (len <= 0) return;
  const uint32_t* w = ws + inst * ws_stride;
  const uint32_t* p0 = w + 2 * h;                 // 2h limbs
  const uint32_t* p2 = w + 4 * h;                 // 2(n-h) limbs
  const uint32_t* pm = w + 6 * h;                 // 2h limbs
  uint32_t* o = out + inst * (int64_t)(2 * n) + k0;
  const int l2 = 2 * (n - h);
  const int s = sgn[2 * inst] * sgn[2 * inst + 1];
  auto t = [&](int k) -> uint64_t {
    uint64_t v = k < 2 * h ? p0[k] : p2[k - 2 * h];
    const int j = k - h;
    if (j >= 0 && j < 2 * h) {
      v += p0[j];
      if (s > 0) v += pm[j];
      else if (s < 0) v += (uint32_t)~pm[j];
    }
    if (j >= 0 && j < l2) v += p2[j];
    if (s < 0) {
      if (k == h) v += 1u;
      if (k >= 3 * h) v += 0xffffffffu;
    }
    return v;
  };
  // thread i: limbs [i Q, i Q + Q) of the chunk; limb k adds the low half of
  // the sum t(k) and the high half of t(k - 1); one round, one scan
  const int j0 = threadIdx.x * kCombQ;
  const int valid = min(kCombQ, max(0, len - j0));
  uint32_t x[kCombQ], y[kCombQ];
  if (VEC) {
    static_assert(kCombQ == 4, "one 16-byte run per thread");
    uint64_t v[4] = {0ull, 0ull, 0ull, 0ull};
    const int k = k0 + j0;
    if (valid > 0) {
      auto add4 = [&](const uint32_t* src, bool inv) {
        const uint4 u = *reinterpret_cast<const uint4*>(src);
        v[0] += inv ? ~u.x : u.x;
        v[1] += inv ? ~u.y : u.y;
        v[2] += inv ? ~u.z : u.z;
        v[3] += inv ? ~u.w : u.w;
      };
      add4(k < 2 * h ? p0 + k : p2 + (k - 2 * h), false);
      const int j = k - h;
      if (j >= 0 && j < 2 * h) {
        add4(p0 + j, false);
        if (s != 0) add4(pm + j, s < 0);
      }
      if (j >= 0 && j < l2) add4(p2 + j, false);
      if (s < 0) {
        if (k == h) v[0] += 1u;
        if (k >= 3 * h) {
          v[0] += 0xffffffffu; v[1] += 0xffffffffu; v[2] += 0xffffffffu; v[3] += 0xffffffffu;
        }
      }
    }
    uint32_t below = (uint32_t)__shfl_up((int)(uint32_t)(v[3] >> 32), 1);
    if (lane_id() == 0) below = (k >= 1 && valid > 0) ? (uint32_t)(t(k - 1) >> 32) : 0u;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      x[i] = (uint32_t)v[i];
      y[i] = i == 0 ? below : (uint32_t)(v[i - 1] >> 32);
    }
  } else {
    uint64_t tv[kCombQ + 1];
#pragma unroll
    for (int i = 0; i <= kCombQ; ++i) {
      const int k = k0 + j0 + i - 1;
      tv[i] = (k >= 0 && k < 2 * n) ? t(k) : 0ull;
    }
#pragma unroll
    for (int i = 0; i < kCombQ; ++i) {
      x[i] = i < valid ? (uint32_t)tv[i + 1] : 0u;
      y[i] = i < valid ? (uint32_t)(tv[i] >> 32) : 0u;
    }
  }
  LimbRun<kCombQ, false> run;
  run.build(x, y, valid);
  uint32_t c;
  const uint32_t cin = wg_carry_scan(run.G, run.P, 0u, scratch, &c);
  run.apply(cin);
  bool ones = true;
  if (VEC) {
    if (valid > 0) *reinterpret_cast<uint4*>(o + j0) = make_uint4(run.s[0], run.s[1], run.s[2], run.s[3]);
#pragma unroll
    for (int i = 0; i < kCombQ; ++i) ones = ones && (i >= valid || run.s[i] == 0xffffffffu);
  } else {
#pragma unroll
    for (int i = 0; i < kCombQ; ++i)
      if (i < valid) {
        o[j0 + i] = run.s[i];
        ones = ones && run.s[i] == 0xffffffffu;
      }
  }
  const bool all = __syncthreads_and(ones);
  if (threadIdx.x == 0) summ[inst * kCombMaxChunks + chunk] = c | (all ? 2u : 0u);
}

// One wave per instance: carries between the chunks of k_kara_combine.
__global__ __launch_bounds__(64) void k_kara_carry(uint32_t* out, const uint32_t* summ, int n) {
  const int64_t inst = blockIdx.x;
  uint32_t* o = out + inst * (int64_t)(2 * n);
  const int lane = lane_id();
  const int nch = (2 * n + kCombChunk - 1) / kCombChunk;
  uint32_t c = 0;
  for (int ch = 0; ch < nch; ++ch) {
    const uint32_t sm = summ[inst * kCombMaxChunks + ch];
    if (c) {  // + 1 at the chunk's first limb
      const int k1 = min((ch + 1) * kCombChunk, 2 * n);
      for (int base = ch * kCombChunk; base < k1; base += 64) {
        const int k = base + lane;
        const uint32_t v = k < k1 ? o[k] : 0u;
        const uint64_t m = __ballot(k < k1 && v != 0xffffffffu);
        if (m) {
          const int f = __ffsll((unsigned long long)m) - 1;  // first limb that absorbs the carry
          if (lane < f) o[k] = 0u;
          else if (lane == f) o[k] = v + 1u;
          break;
        }
        if (k < k1) o[k] = 0u;
      }
    }
    c = (sm & 1u) | ((sm >> 1) & c);
  }
}

size_t kara_ws_bytes(int n, int64_t batch) {
  const int h = (n + 1) / 2;
  return (size_t)batch * (10 * (size_t)h + 16) * 4 + (size_t)batch * 8 +
         (size_t)batch * kCombMaxChunks * 4 + 256;
}

int launch_mul_kara(uint32_t* out, const uint32_t* a, const uint32_t* b, int64_t n, int64_t batch,
                    void* ws_v, MfmaCfg cfg, hipStream_t s) {
  const int h = (int)((n + 1) / 2);
  const int64_t ws_stride = 10 * (int64_t)h + 16;
  uint32_t* ws = reinterpret_cast<uint32_t*>(ws_v);
  int32_t* sgn = reinterpret_cast<int32_t*>(ws + batch * ws_stride);
  uint32_t* summ = reinterpret_cast<uint32_t*>(sgn + 2 * batch);
  if (h > kKaraQ * 1024) return BIGINT_EUNSUPPORTED;
  const int nch = (int)((2 * n + kCombChunk - 1) / kCombChunk);
  if (nch > kCombMaxChunks) return BIGINT_EUNSUPPORTED;
  // |a0 - a1| at ws[0..h), |b1 - b0| at ws[h..2h), signs
  const int T = (int)((cdiv(h, kKaraQ) + 63) / 64 * 64);
  // 16-byte runs: n a multiple of 8 (h, n - h, 2h, 3h multiples of 4) and
  // aligned buffers (the workspace stride 10h + 16 keeps each instance's
  // parts aligned)
  const bool vec = n % 8 == 0 && (uintptr_t)a % 16 == 0 && (uintptr_t)b % 16 == 0 &&
                   (uintptr_t)out % 16 == 0 && (uintptr_t)ws % 16 == 0;
  if (vec)
    hipLaunchKernelGGL(k_kara_diff<true>, dim3((unsigned)batch, 2), dim3(T), 0, s, ws, ws_stride,
                       sgn, a, b, (int)n, h);
  else
    hipLaunchKernelGGL(k_kara_diff<false>, dim3((unsigned)batch, 2), dim3(T), 0, s, ws, ws_stride,
                       sgn, a, b, (int)n, h);
  BI_LAUNCH_CHECK();
  // p0 = a0 b0, p2 = a1 b1, pm = |a0 - a1| |b1 - b0|
  KaraJobs J;
  J.j[0] = KaraJob{ws + 2 * h, ws_stride, a, n, b, n, h, h};
  J.j[1] = KaraJob{ws + 4 * h, ws_stride, a + h, n, b + h, n, (int)n - h, (int)n - h};
  J.j[2] = KaraJob{ws + 6 * h, ws_stride, ws, ws_stride, ws + h, ws_stride, h, h};
  const size_t lds = cfg.dw == 8 ? mfma::lds_bytes<8>(h, h, cfg.waves, cfg.P)
                                 : mfma::lds_bytes<7>(h, h, cfg.waves, cfg.P);
  if (lds > 163840) return BIGINT_EUNSUPPORTED;
  const dim3 gd((unsigned)batch, 3), bd(64 * cfg.waves);
#define BI_KARA_LAUNCH(DW, PP)                                                                    \
  do {                                                                                            \
    BI_HIP(hipFuncSetAttribute((const void*)k_kara_mul<DW, PP>,                                   \
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));            \
    hipLaunchKernelGGL((k_kara_mul<DW, PP>), gd, bd, lds, s, J);                                  \
  } while (0)
  if (cfg.dw == 8) {
    if (cfg.P == 4) BI_KARA_LAUNCH(8, 4);
    else if (cfg.P == 8) BI_KARA_LAUNCH(8, 8);
    else BI_KARA_LAUNCH(8, 16);
  } else {
    if (cfg.P == 4) BI_KARA_LAUNCH(7, 4);
    else if (cfg.P == 8) BI_KARA_LAUNCH(7, 8);
    else BI_KARA_LAUNCH(7, 16);
  }
#undef BI_KARA_LAUNCH
  BI_LAUNCH_CHECK();
  // the sum
  if (vec)
    hipLaunchKernelGGL(k_kara_combine<true>, dim3((unsigned)batch, nch), dim3(1024), 0, s, out, ws,
                       ws_stride, sgn, summ, (int)n, h);
  else
    hipLaunchKernelGGL(k_kara_combine<false>, dim3((unsigned)batch, nch), dim3(1024), 0, s, out,
                       ws, ws_stride, sgn, summ, (int)n, h);
  BI_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_kara_carry, dim3((unsigned)batch), dim3(64), 0, s, out, summ, (int)n);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

}  // namespace bi
