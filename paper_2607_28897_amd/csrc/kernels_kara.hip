// kernels_kara.hip -- one Karatsuba level over the MFMA-split multiply.
//
// With h = ceil(n/2), a = a1 B^h + a0 and b = b1 B^h + b0 (a0, b0: h limbs;
// a1, b1: n - h limbs):
//   a b = p2 B^(2h) + (p0 + p2 + s pm) B^h + p0,
//   p0 = a0 b0, p2 = a1 b1, pm = |a0 - a1| |b1 - b0|,
//   s = sign(a0 - a1) sign(b1 - b0),
// since a0 b1 + a1 b0 = (a0 - a1)(b1 - b0) + a0 b0 + a1 b1.  Three products
// of half the size replace one: 3/4 of the multiply-accumulates, for two
// linear passes before and three after.
#include "internal.hpp"
#include "dev_addsub.hpp"
#include "dev_mul_mfma.hpp"

namespace bi {

// d = |x - y| over n limbs and sgn = sign(x - y) (x: nx limbs, y: ny limbs,
// zero-extended; n <= 16 * blockDim.x).  Both differences are formed in the
// same pass; the borrow out of x - y picks one.  blockIdx.y = 0: x = a0,
// y = a1; = 1: x = b1, y = b0.
constexpr int kKaraQ = 16;

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
#pragma unroll
  for (int i = 0; i < kKaraQ; ++i) {
    const int j = j0 + i;
    const uint32_t xa = x[max(min(j, nx - 1), 0)], ya = y[max(min(j, ny - 1), 0)];
    xv[i] = (i < valid && j < nx) ? xa : 0u;
    yv[i] = (i < valid && j < ny) ? ya : 0u;
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
#pragma unroll
  for (int i = 0; i < kKaraQ; ++i)
    if (i < valid) d[j0 + i] = borrow ? r2.s[i] : r1.s[i];
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

// out (2n limbs) = p0 + p2 B^(2h) + (p0 + p2 + s pm) B^h.
__global__ __launch_bounds__(1024) void k_kara_combine(uint32_t* out, const uint32_t* ws,
                                                       int64_t ws_stride, const int32_t* sgn,
                                                       int n, int h) {
  __shared__ uint32_t scratch[32];
  const int64_t inst = blockIdx.x;
  const uint32_t* w = ws + inst * ws_stride;
  const uint32_t* p0 = w + 2 * h;                 // 2h limbs
  const uint32_t* p2 = w + 4 * h;                 // 2(n-h) limbs
  const uint32_t* pm = w + 6 * h;                 // 2h limbs
  uint32_t* M = const_cast<uint32_t*>(w) + 8 * h; // 2h+1 limbs
  uint32_t* o = out + inst * (int64_t)(2 * n);
  const int l2 = 2 * (n - h);
  const int s = sgn[2 * inst] * sgn[2 * inst + 1];
  {  // M = p0 + p2
    auto X = [&](int j) -> uint32_t { return j < 2 * h ? p0[j] : 0u; };
    auto Y = [&](int j) -> uint32_t { return j < l2 ? p2[min(j, l2 - 1)] : 0u; };
    wg_addsub<16, false>(M, 2 * h + 1, X, Y, 0u, scratch);
  }
  if (s != 0) {  // M += s pm (the result is a0 b1 + a1 b0 >= 0)
    auto X = [&](int j) -> uint32_t { return M[j]; };
    auto Y = [&](int j) -> uint32_t { return j < 2 * h ? pm[j] : 0u; };
    if (s > 0)
      wg_addsub<16, false>(M, 2 * h + 1, X, Y, 0u, scratch);
    else
      wg_addsub<16, true>(M, 2 * h + 1, X, Y, 0u, scratch);
  }
  // o[0..h) = p0[0..h); o[h..2n) = (p0 B^0 + p2 B^(2h))[h..2n) + M
  for (int j = threadIdx.x; j < h; j += blockDim.x) o[j] = p0[j];
  auto X = [&](int j) -> uint32_t {
    const int k = h + j;
    return k < 2 * h ? p0[k] : p2[min(k - 2 * h, l2 - 1)];
  };
  auto Y = [&](int j) -> uint32_t { return j <= 2 * h ? M[min(j, 2 * h)] : 0u; };
  wg_addsub<16, false>(o + h, 2 * n - h, X, Y, 0u, scratch);
}

size_t kara_ws_bytes(int n, int64_t batch) {
  const int h = (n + 1) / 2;
  return (size_t)batch * (10 * (size_t)h + 16) * 4 + (size_t)batch * 8 + 256;
}

int launch_mul_kara(uint32_t* out, const uint32_t* a, const uint32_t* b, int64_t n, int64_t batch,
                    void* ws_v, MfmaCfg cfg, hipStream_t s) {
  const int h = (int)((n + 1) / 2);
  const int64_t ws_stride = 10 * (int64_t)h + 16;
  uint32_t* ws = reinterpret_cast<uint32_t*>(ws_v);
  int32_t* sgn = reinterpret_cast<int32_t*>(ws + batch * ws_stride);
  if (h > kKaraQ * 1024) return BIGINT_EUNSUPPORTED;
  // |a0 - a1| at ws[0..h), |b1 - b0| at ws[h..2h), signs
  const int T = (int)((cdiv(h, kKaraQ) + 63) / 64 * 64);
  hipLaunchKernelGGL(k_kara_diff, dim3((unsigned)batch, 2), dim3(T), 0, s, ws, ws_stride, sgn, a,
                     b, (int)n, h);
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
  hipLaunchKernelGGL(k_kara_combine, dim3((unsigned)batch), dim3(1024), 0, s, out, ws, ws_stride,
                     sgn, (int)n, h);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

}  // namespace bi
