// kernels.hip -- gfx950 kernels of the batched big-integer library and their
// host launchers.
#include "internal.hpp"
#include "dev_addsub.hpp"
#include "dev_mul_mfma.hpp"
#include "dev_mul_plain.hpp"

namespace bi {

// ============================================================================
// add / sub: one work-group per instance, Q consecutive limbs per thread
// loaded with 16-byte vector loads (Section 5.1: badd copies the operands
// from global memory into registers, baddReg scans the per-thread carries).
// ============================================================================
template <int Q, bool SUB, bool VEC>
__global__ __launch_bounds__(1024) void k_addsub(uint32_t* out, uint32_t* cout, const uint32_t* a,
                                                 const uint32_t* b, int n) {
  __shared__ uint32_t scratch[32];
  const int64_t inst = blockIdx.x;
  const uint32_t* pa = a + inst * n;
  const uint32_t* pb = b + inst * n;
  uint32_t* po = out + inst * n;
  const int j0 = threadIdx.x * Q;
  const int valid = min(Q, max(0, n - j0));
  LimbRun<Q, SUB> run;
  run.start();
  if (VEC && valid == Q) {
#pragma unroll
    for (int i = 0; i < Q; i += 4) {
      const uint4 va = *reinterpret_cast<const uint4*>(pa + j0 + i);
      const uint4 vb = *reinterpret_cast<const uint4*>(pb + j0 + i);
      run.set(i, va.x, vb.x, true);
      run.set(i + 1, va.y, vb.y, true);
      run.set(i + 2, va.z, vb.z, true);
      run.set(i + 3, va.w, vb.w, true);
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const bool ok = i < valid;
      run.set(i, ok ? pa[j0 + i] : 0u, ok ? pb[j0 + i] : 0u, ok);
    }
  }
  run.finish();
  uint32_t total;
  const uint32_t c = wg_carry_scan(run.G, run.P, 0u, scratch, &total);
  run.apply(c);
  if (VEC && valid == Q) {
#pragma unroll
    for (int i = 0; i < Q; i += 4)
      *reinterpret_cast<uint4*>(po + j0 + i) =
          make_uint4(run.s[i], run.s[i + 1], run.s[i + 2], run.s[i + 3]);
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (i < valid) po[j0 + i] = run.s[i];
  }
  if (cout && threadIdx.x == 0) cout[inst] = total;
}

template <bool SUB>
__global__ __launch_bounds__(1024) void k_addsub_rounds(uint32_t* out, uint32_t* cout,
                                                        const uint32_t* a, const uint32_t* b, int n) {
  __shared__ uint32_t scratch[32];
  const int64_t inst = blockIdx.x;
  const uint32_t* pa = a + inst * n;
  const uint32_t* pb = b + inst * n;
  auto X = [&](int j) -> uint32_t { return pa[j]; };
  auto Y = [&](int j) -> uint32_t { return pb[j]; };
  const uint32_t c = wg_addsub<16, SUB>(out + inst * n, n, X, Y, 0u, scratch);
  if (cout && threadIdx.x == 0) cout[inst] = c;
}

template <int Q, bool SUB>
static int launch_addsub_q(uint32_t* out, uint32_t* cout, const uint32_t* a, const uint32_t* b,
                           int64_t n, int64_t batch, hipStream_t s) {
  const int T = (int)((cdiv(n, Q) + 63) / 64 * 64);
  const bool vec = (n % 4 == 0) && ((uintptr_t)a % 16 == 0) && ((uintptr_t)b % 16 == 0) &&
                   ((uintptr_t)out % 16 == 0);
  if (vec)
    hipLaunchKernelGGL((k_addsub<Q, SUB, true>), dim3((unsigned)batch), dim3(T), 0, s, out, cout, a,
                       b, (int)n);
  else
    hipLaunchKernelGGL((k_addsub<Q, SUB, false>), dim3((unsigned)batch), dim3(T), 0, s, out, cout,
                       a, b, (int)n);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

// ---- several instances per wave (the paper's ipb) for short operands --------
// Lanes [k L, (k+1) L) of a wave hold instance k of that wave (L = ceil(n/Q)
// lanes of Q limbs; ipw = 64 / L instances per wave, 4 waves per
// work-group).  The carry scan is segmented: the generate and propagate bits
// of each instance's last lane are left out of the ballots, so no carry
// crosses into the next instance, and that lane's own carry out (the
// instance's) comes from its run summary and its carry in.  STEPS = 1: one
// addition (or subtraction); STEPS = 6: the 6-Add chain a+b+a+b+a+b+a with
// the carries out counted.
template <int Q, bool SUB, int STEPS, bool VEC>
__global__ __launch_bounds__(256) void k_addsub_ipb(uint32_t* out, uint32_t* cout, const uint32_t* a,
                                                    const uint32_t* b, int n, int L, int ipw,
                                                    int64_t batch) {
  const int lane = lane_id();
  const int k = lane / L, li = lane - k * L;
  const int64_t inst = ((int64_t)blockIdx.x * 4 + wave_id()) * ipw + k;
  const bool live = k < ipw && inst < batch;
  const int j0 = li * Q;
  const int valid = live ? min(Q, max(0, n - j0)) : 0;
  const int64_t base = live ? inst * (int64_t)n : 0;
  uint32_t av[Q], bv[Q], x[Q];
  if (VEC && valid == Q) {
#pragma unroll
    for (int i = 0; i < Q; i += 4) {
      const uint4 va = *reinterpret_cast<const uint4*>(a + base + j0 + i);
      const uint4 vb = *reinterpret_cast<const uint4*>(b + base + j0 + i);
      av[i] = va.x; av[i + 1] = va.y; av[i + 2] = va.z; av[i + 3] = va.w;
      bv[i] = vb.x; bv[i + 1] = vb.y; bv[i + 2] = vb.z; bv[i + 3] = vb.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int64_t jj = base + min(j0 + i, n - 1);
      av[i] = i < valid ? a[jj] : 0u;
      bv[i] = i < valid ? b[jj] : 0u;
    }
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) x[i] = av[i];
  const bool last = live && li == L - 1;
  uint32_t total = 0;
#pragma unroll
  for (int step = 0; step < STEPS; ++step) {
    LimbRun<Q, SUB> run;
    run.build(x, (step & 1) ? av : bv, valid);
    const WaveCarry w = wave_carry_masks(run.G && !last, run.P && !last);
    const uint32_t c = wave_carry_in(w, 0u);
    run.apply(c);
#pragma unroll
    for (int i = 0; i < Q; ++i) x[i] = run.s[i];
    total += (uint32_t)(run.G | (run.P & (c != 0u)));
  }
  if (VEC && valid == Q) {
#pragma unroll
    for (int i = 0; i < Q; i += 4)
      *reinterpret_cast<uint4*>(out + base + j0 + i) = make_uint4(x[i], x[i + 1], x[i + 2], x[i + 3]);
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (i < valid) out[base + j0 + i] = x[i];
  }
  if (cout && last) cout[inst] = total;
}

constexpr int kIpbQ = 4;
constexpr int kIpbMax = 64 * kIpbQ;   // limbs: one instance fills at most one wave

template <bool SUB, int STEPS>
static int launch_addsub_ipb(uint32_t* out, uint32_t* cout, const uint32_t* a, const uint32_t* b,
                             int64_t n, int64_t batch, hipStream_t s) {
  const int L = (int)cdiv(n, kIpbQ);
  const int ipw = 64 / L;
  const int64_t per_wg = 4 * (int64_t)ipw;
  const dim3 gd((unsigned)((batch + per_wg - 1) / per_wg)), bd(256);
  const bool vec = (n % 4 == 0) && ((uintptr_t)a % 16 == 0) && ((uintptr_t)b % 16 == 0) &&
                   ((uintptr_t)out % 16 == 0);
  if (vec)
    hipLaunchKernelGGL((k_addsub_ipb<kIpbQ, SUB, STEPS, true>), gd, bd, 0, s, out, cout, a, b,
                       (int)n, L, ipw, batch);
  else
    hipLaunchKernelGGL((k_addsub_ipb<kIpbQ, SUB, STEPS, false>), gd, bd, 0, s, out, cout, a, b,
                       (int)n, L, ipw, batch);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

template <bool SUB>
static int launch_addsub_t(uint32_t* out, uint32_t* cout, const uint32_t* a, const uint32_t* b,
                           int64_t n, int64_t batch, hipStream_t s) {
  // up to 256 limbs: several instances per wave; up to 2048 limbs: 256
  // threads per instance; above: 1024 threads, which keeps more loads in
  // flight per CU (measured: 5.6 against 4.4 TB/s at 8192 limbs), with 4..32
  // limbs each
  if (n <= kIpbMax) return launch_addsub_ipb<SUB, 1>(out, cout, a, b, n, batch, s);
  if (n <= 1024) return launch_addsub_q<4, SUB>(out, cout, a, b, n, batch, s);
  if (n <= 2048) return launch_addsub_q<8, SUB>(out, cout, a, b, n, batch, s);
  if (n <= 4096) {
    // 1024-thread groups sit two per CU; when the batch needs a second round
    // of them but four 512-thread groups per CU hold it at once, the smaller
    // groups finish in one round (1024 x 2^17 bits: 13.0 -> 11.8 us)
    const int64_t cus = num_cus();
    if (batch > 2 * cus && batch <= 4 * cus) return launch_addsub_q<8, SUB>(out, cout, a, b, n, batch, s);
    return launch_addsub_q<4, SUB>(out, cout, a, b, n, batch, s);
  }
  if (n <= 8192) return launch_addsub_q<8, SUB>(out, cout, a, b, n, batch, s);
  if (n <= 16384) return launch_addsub_q<16, SUB>(out, cout, a, b, n, batch, s);
  if (n <= 32768) return launch_addsub_q<32, SUB>(out, cout, a, b, n, batch, s);
  // beyond 1024 threads x 32 limbs: rounds of the work-group add, carry chained
  hipLaunchKernelGGL((k_addsub_rounds<SUB>), dim3((unsigned)batch), dim3(1024), 0, s, out, cout, a,
                     b, (int)n);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

int launch_addsub(bool sub, uint32_t* out, uint32_t* cout, const uint32_t* a, const uint32_t* b,
                  int64_t n, int64_t batch, hipStream_t s) {
  return sub ? launch_addsub_t<true>(out, cout, a, b, n, batch, s)
             : launch_addsub_t<false>(out, cout, a, b, n, batch, s);
}

// ============================================================================
// plain u64 multiply: one work-group per instance
// ============================================================================
constexpr int kPlainQ = 4;
constexpr int kPlainR = 4;

template <int Q, int R>
__global__ __launch_bounds__(1024) void k_mul_plain(uint32_t* out, const uint32_t* a, int na,
                                                    const uint32_t* b, int nb) {
  extern __shared__ uint64_t sm64[];
  const int64_t inst = blockIdx.x;
  wg_mul_plain<Q, R>(out + inst * (int64_t)(na + nb), a + inst * (int64_t)na, na,
                     b + inst * (int64_t)nb, nb, sm64);
}

template <int Q, int R, int S>
__global__ __launch_bounds__(1024) void k_mul_plain_split(uint32_t* out, const uint32_t* a, int na,
                                                          const uint32_t* b, int nb) {
  extern __shared__ uint64_t sm64[];
  const int64_t inst = blockIdx.x;
  wg_mul_plain_split<Q, R, S>(out + inst * (int64_t)(na + nb), a + inst * (int64_t)na, na,
                              b + inst * (int64_t)nb, nb, sm64);
}

size_t plain_lds(int na, int nb) { return plain_lds_bytes(na, nb); }

static int plain_threads(int na, int nb) {
  const int K = (na + 1) / 2 + (nb + 1) / 2;
  const int NBLK = (K + kPlainQ - 1) / kPlainQ;
  int T = (int)((cdiv(NBLK, kPlainR) + 63) / 64 * 64);
  return T < 64 ? 64 : T;
}

// Parts per product for the split kernel.  Below 256 threads a work-group
// leaves SIMDs of its CU idle: one wave of its own keeps a SIMD's VALU busy,
// so more waves on the same SIMDs gain nothing.  When the batch leaves SIMDs
// without waves, every block's common range is cut into 2 or 4 parts, up to
// one wave per SIMD of the work-group's CU (measured: 64 pairs of 1024
// limbs: 0.131 -> 0.044 ms with 4 parts, 0.052 ms with 8 parts on two waves
// per SIMD; 4096-limb products on 256 threads got 7% slower with 4 parts).
static int plain_parts(int na, int nb, int64_t batch, int T) {
  const int64_t simds = 4 * (int64_t)num_cus();
  int S = 1;
  while (S < 4 && batch * (T / 64) * S * 2 <= simds && T * S * 2 <= 256 &&
         plain_split_lds_bytes(na, nb, S * 2, T, kPlainQ) <= 163840)
    S *= 2;
  return S;
}

template <int S>
static int launch_mul_plain_split(uint32_t* out, const uint32_t* a, int64_t na, const uint32_t* b,
                                  int64_t nb, int64_t batch, int T, hipStream_t s) {
  const size_t lds = plain_split_lds_bytes((int)na, (int)nb, S, T, kPlainQ);
  BI_HIP(hipFuncSetAttribute((const void*)k_mul_plain_split<kPlainQ, kPlainR, S>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_mul_plain_split<kPlainQ, kPlainR, S>), dim3((unsigned)batch), dim3(T * S),
                     lds, s, out, a, (int)na, b, (int)nb);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

int launch_mul_plain(uint32_t* out, const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb,
                     int64_t batch, hipStream_t s) {
  const int T = plain_threads((int)na, (int)nb);
  if (T > 1024) return BIGINT_EUNSUPPORTED;
  switch (plain_parts((int)na, (int)nb, batch, T)) {
    case 2: return launch_mul_plain_split<2>(out, a, na, b, nb, batch, T, s);
    case 4: return launch_mul_plain_split<4>(out, a, na, b, nb, batch, T, s);
    default: break;
  }
  const size_t lds = plain_lds((int)na, (int)nb);
  BI_HIP(hipFuncSetAttribute((const void*)k_mul_plain<kPlainQ, kPlainR>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_mul_plain<kPlainQ, kPlainR>), dim3((unsigned)batch), dim3(T), lds, s, out,
                     a, (int)na, b, (int)nb);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

// ============================================================================
// MFMA-split multiply: one work-group per instance
// ============================================================================
// out instance i = a_i * b_i mod B^nout (nout = na + nb: the whole product);
// lead != 0: the LDS holds every strip's limbs 0-1 (see wg_mul_mfma)
template <int DW, int P, int TS>
__global__ __launch_bounds__(512) void k_mul_mfma(uint32_t* out, int32_t* coef, const uint32_t* a,
                                                  int na, const uint32_t* b, int nb, int nout, int lead) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int64_t inst = blockIdx.x;
  const int K = mfma::ndigits(na) + mfma::ndigits(nb) - 1;
  mfma::wg_mul_mfma<DW, P, TS>(out ? out + inst * (int64_t)nout : nullptr,
                           coef ? coef + inst * (int64_t)K : nullptr, a + inst * (int64_t)na, na,
                           b + inst * (int64_t)nb, nb, smem, nout, 0, 0, 1, nullptr, lead != 0);
}

// LDS of the work-group kernel (waves == 1, one wave per instance, is sized
// as its 4-wave fallback, which covers it)
size_t mfma_lds(int na, int nb, MfmaCfg cfg) {
  if (cfg.waves == 1) cfg.waves = 4;
  if (cfg.tile == 32) return mfma::lds_bytes<8, 32>(na, nb, cfg.waves, cfg.P);
  return cfg.dw == 8 ? mfma::lds_bytes<8>(na, nb, cfg.waves, cfg.P)
                     : mfma::lds_bytes<7>(na, nb, cfg.waves, cfg.P);
}

template <int DW, int P, int TS = 16>
static int launch_mfma_p(uint32_t* out, int32_t* coef, const uint32_t* a, int64_t na,
                         const uint32_t* b, int64_t nb, int64_t batch, int waves, int nout,
                         hipStream_t s) {
  size_t lds = mfma::lds_bytes<DW, TS>((int)na, (int)nb, waves, P);
  if (lds > 163840) return BIGINT_EUNSUPPORTED;
  // keep the strips' limbs 0-1 in LDS for the closing scan (no read-back from
  // global memory) where the extra 8 bytes per strip fit without costing a
  // resident work-group per CU
  const size_t lds_lead = mfma::lds_bytes<DW, TS>((int)na, (int)nb, waves, P, true);
  const int lead = DW == 8 && coef == nullptr && lds_lead <= 163840 && 163840 / lds_lead == 163840 / lds;
  if (lead) lds = lds_lead;
  BI_HIP(hipFuncSetAttribute((const void*)k_mul_mfma<DW, P, TS>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_mul_mfma<DW, P, TS>), dim3((unsigned)batch), dim3(64 * waves), lds, s, out,
                     coef, a, (int)na, b, (int)nb, nout, lead);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

template <int DW>
static int launch_mfma_dw(uint32_t* out, int32_t* coef, const uint32_t* a, int64_t na,
                          const uint32_t* b, int64_t nb, int64_t batch, MfmaCfg cfg, int nout,
                          hipStream_t s) {
  if constexpr (DW == 8) {
    if (cfg.tile == 32) {
      switch (cfg.P) {
        case 8: return launch_mfma_p<8, 8, 32>(out, coef, a, na, b, nb, batch, cfg.waves, nout, s);
        case 16: return launch_mfma_p<8, 16, 32>(out, coef, a, na, b, nb, batch, cfg.waves, nout, s);
        case 32: return launch_mfma_p<8, 32, 32>(out, coef, a, na, b, nb, batch, cfg.waves, nout, s);
        default: return BIGINT_EINVAL;
      }
    }
  }
  switch (cfg.P) {
    case 4: return launch_mfma_p<DW, 4>(out, coef, a, na, b, nb, batch, cfg.waves, nout, s);
    case 8: return launch_mfma_p<DW, 8>(out, coef, a, na, b, nb, batch, cfg.waves, nout, s);
    case 16: return launch_mfma_p<DW, 16>(out, coef, a, na, b, nb, batch, cfg.waves, nout, s);
    default: return BIGINT_EINVAL;
  }
}

// ---- fewer products than CUs: each product's bands split over work-groups ----
// Part p of instance i (blockIdx.x, blockIdx.y) computes a contiguous run of
// the product's bands of about 1/nparts of its cost (4 strips per band, 4
// waves) and writes its strips' carry words to ws[i * wstride + w]; a second
// launch (k_mul_mfma_close) then runs the closing strip carry scan of every
// instance.  The bytes are those of one work-group per instance.
constexpr int kSplitP = 4, kSplitWaves = 4;

template <int DW>
__global__ __launch_bounds__(64 * kSplitWaves) void k_mul_mfma_part(uint32_t* out, const uint32_t* a,
                                                                   int na, const uint32_t* b, int nb,
                                                                   int nout, uint64_t* ws, int wstride,
                                                                   int nparts) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int64_t inst = blockIdx.y;
  mfma::wg_mul_mfma<DW, kSplitP>(out + inst * (int64_t)nout, nullptr, a + inst * (int64_t)na, na,
                                 b + inst * (int64_t)nb, nb, smem, nout, 0, (int)blockIdx.x, nparts,
                                 ws + inst * (int64_t)wstride);
}

template <int DW>
__global__ __launch_bounds__(1024) void k_mul_mfma_close(uint32_t* out, int na, int nb, int nout,
                                                         const uint64_t* ws, int wstride) {
  __shared__ uint32_t scratch[32];
  const int64_t inst = blockIdx.x;
  const mfma::Geo g = mfma::make_geo<DW>(na, nb, nout);
  mfma::close_strips<DW>(out + inst * (int64_t)nout, g, ws + inst * (int64_t)wstride, 0, scratch);
}

// Parts per instance for an na x nb product (mod B^nout) over `batch` instances (1:
// no split): enough work-groups for every CU once, at least four bands per
// part, at least four parts and at least 32 bands (128 strips): with two
// parts, or four thin ones, the parts' 4-strip bands on 4 waves lose more
// than the extra CUs gain (128 products of 2^19 bits 0.54 -> 0.70 ms, 64 of
// 2^15 bits 17 -> 31 us, one 4096-limb product mod B^n 36 -> 37 us); with
// four or more, 2^19 bits: 1 or 4 products 0.52 -> 0.127 ms, 16 products
// 0.52 -> 0.19, 64 products 0.53 -> 0.39; 2^17 bits, 1 or 16 products
// 0.053 -> 0.041; products mod B^n of 2^19 bits, 1 or 16: 0.29 -> 0.115);
// *wstride = strips per instance (carry words of workspace each).
int mul_mfma_split_parts(int na, int nb, int nout, int64_t batch, int dw, int* wstride) {
  const int W = dw == 8 ? mfma::make_geo<8>(na, nb, nout).W : mfma::make_geo<7>(na, nb, nout).W;
  *wstride = W;
  const int R = num_cus();
  if (batch <= 0 || batch >= R) return 1;
  const size_t lds = dw == 8 ? mfma::lds_bytes<8>(na, nb, kSplitWaves, kSplitP)
                             : mfma::lds_bytes<7>(na, nb, kSplitWaves, kSplitP);
  if (lds > 163840) return 1;
  const int NB = (W + kSplitP - 1) / kSplitP;
  if (NB < 32) return 1;
  const int k = (int)std::min<int64_t>((R + batch - 1) / batch, NB / 4);
  return k >= 4 ? k : 1;
}

// The split configuration for one instance of a ragged segment: strips
// (carry words) and the part kernel's LDS.
void ragged_split_geo(int na, int nb, int dw, int* strips, size_t* lds) {
  if (dw == 8) {
    *strips = mfma::make_geo<8>(na, nb, na + nb).W;
    *lds = mfma::lds_bytes<8>(na, nb, kSplitWaves, kSplitP);
  } else {
    *strips = mfma::make_geo<7>(na, nb, na + nb).W;
    *lds = mfma::lds_bytes<7>(na, nb, kSplitWaves, kSplitP);
  }
}

int launch_mul_mfma_split(uint32_t* out, const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb,
                          int nout, int64_t batch, int dw, int nparts, uint64_t* ws, int wstride,
                          hipStream_t s) {
  const int W = wstride;
  const unsigned close_threads = (unsigned)std::min(1024, (W + 63) / 64 * 64);
  const dim3 gp((unsigned)nparts, (unsigned)batch);
  if (dw == 8) {
    const size_t lds = mfma::lds_bytes<8>((int)na, (int)nb, kSplitWaves, kSplitP);
    BI_HIP(hipFuncSetAttribute((const void*)k_mul_mfma_part<8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    hipLaunchKernelGGL(k_mul_mfma_part<8>, gp, dim3(64 * kSplitWaves), lds, s, out, a, (int)na, b,
                       (int)nb, nout, ws, wstride, nparts);
    BI_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mul_mfma_close<8>, dim3((unsigned)batch), dim3(close_threads), 0, s, out,
                       (int)na, (int)nb, nout, ws, wstride);
  } else {
    const size_t lds = mfma::lds_bytes<7>((int)na, (int)nb, kSplitWaves, kSplitP);
    BI_HIP(hipFuncSetAttribute((const void*)k_mul_mfma_part<7>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    hipLaunchKernelGGL(k_mul_mfma_part<7>, gp, dim3(64 * kSplitWaves), lds, s, out, a, (int)na, b,
                       (int)nb, nout, ws, wstride, nparts);
    BI_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mul_mfma_close<7>, dim3((unsigned)batch), dim3(close_threads), 0, s, out,
                       (int)na, (int)nb, nout, ws, wstride);
  }
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

// coef != nullptr (raw coefficients) is served with 7-bit digits only.
// nout < 0: the whole na+nb limbs; else the product mod B^nout per instance.
// Small operands: one wave per instance, kWaveInst instances per work-group
// (cfg.waves == 1); every phase runs inside the wave (mfma::wave_mul_mfma).
constexpr int kWaveInst = 4;

template <int P>
__global__ __launch_bounds__(64 * kWaveInst) void k_mul_mfma_wave(uint32_t* out, const uint32_t* a,
                                                                  int na, const uint32_t* b, int nb,
                                                                  int nout, int64_t batch,
                                                                  int wave_lds) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int64_t inst = (int64_t)blockIdx.x * kWaveInst + wave_id();
  if (inst >= batch) return;   // the whole wave: no work-group barrier follows
  mfma::wave_mul_mfma<P>(out + inst * (int64_t)nout, a + inst * (int64_t)na, na,
                         b + inst * (int64_t)nb, nb, smem + (size_t)wave_id() * wave_lds, nout);
}

bool mfma_wave_fits(int64_t na, int64_t nb) {
  return na + nb <= 64 * mfma::strip_limbs<8>() &&
         (size_t)kWaveInst * mfma::wave_lds_bytes((int)na, (int)nb) <= 163840;
}

static int launch_mfma_wave(uint32_t* out, const uint32_t* a, int64_t na, const uint32_t* b,
                            int64_t nb, int64_t batch, int P, int nout, hipStream_t s) {
  const int wl = (int)mfma::wave_lds_bytes((int)na, (int)nb);
  const size_t lds = (size_t)kWaveInst * wl;
  const dim3 gd((unsigned)((batch + kWaveInst - 1) / kWaveInst)), bd(64 * kWaveInst);
  if (P == 4) {
    BI_HIP(hipFuncSetAttribute((const void*)k_mul_mfma_wave<4>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_mul_mfma_wave<4>, gd, bd, lds, s, out, a, (int)na, b, (int)nb, nout,
                       batch, wl);
  } else {
    BI_HIP(hipFuncSetAttribute((const void*)k_mul_mfma_wave<8>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_mul_mfma_wave<8>, gd, bd, lds, s, out, a, (int)na, b, (int)nb, nout,
                       batch, wl);
  }
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

int launch_mul_mfma(uint32_t* out, int32_t* coef, const uint32_t* a, int64_t na,
                    const uint32_t* b, int64_t nb, int64_t batch, MfmaCfg cfg, hipStream_t s,
                    int nout) {
  if (nout < 0 || nout > na + nb) nout = (int)(na + nb);
  if (cfg.waves == 1) {
    if (cfg.dw == 8 && coef == nullptr && mfma_wave_fits(na, nb))
      return launch_mfma_wave(out, a, na, b, nb, batch, cfg.P == 4 ? 4 : 8, nout, s);
    cfg.waves = 4;   // otherwise the work-group kernel
  }
  if (cfg.dw == 8 && coef == nullptr)
    return launch_mfma_dw<8>(out, nullptr, a, na, b, nb, batch, cfg, nout, s);
  if (cfg.dw != 7 && cfg.dw != 8) return BIGINT_EINVAL;
  cfg.tile = 16;   // raw coefficients and 7-bit digits: 16x16 tiles
  return launch_mfma_dw<7>(out, coef, a, na, b, nb, batch, cfg, coef ? (int)(na + nb) : nout, s);
}

// ============================================================================
// fused workloads of the evaluation: 6-Add and Poly
// ============================================================================
// 6-Add: ((((((a+b)+a)+b)+a)+b)+a) mod B^n with the operands and the running
// sum in registers: one HBM pass (read a, b; write the result), six
// work-group carry scans.  ovf[i] = how many of the six additions carried out.
template <int Q, bool VEC>
__global__ __launch_bounds__(1024) void k_add6(uint32_t* out, uint32_t* ovf, const uint32_t* a,
                                               const uint32_t* b, int n) {
  __shared__ uint32_t scratch[32];
  const int64_t inst = blockIdx.x;
  const uint32_t* pa = a + inst * n;
  const uint32_t* pb = b + inst * n;
  uint32_t* po = out + inst * n;
  const int j0 = threadIdx.x * Q;
  const int valid = min(Q, max(0, n - j0));
  uint32_t av[Q], bv[Q], x[Q];
  if (VEC && valid == Q) {
#pragma unroll
    for (int i = 0; i < Q; i += 4) {
      const uint4 va = *reinterpret_cast<const uint4*>(pa + j0 + i);
      const uint4 vb = *reinterpret_cast<const uint4*>(pb + j0 + i);
      av[i] = va.x; av[i + 1] = va.y; av[i + 2] = va.z; av[i + 3] = va.w;
      bv[i] = vb.x; bv[i + 1] = vb.y; bv[i + 2] = vb.z; bv[i + 3] = vb.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int jj = min(j0 + i, n - 1);
      av[i] = i < valid ? pa[jj] : 0u;
      bv[i] = i < valid ? pb[jj] : 0u;
    }
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) x[i] = av[i];
  uint32_t total = 0;
#pragma unroll
  for (int step = 0; step < 6; ++step) {
    LimbRun<Q, false> run;
    run.build(x, (step & 1) ? av : bv, valid);
    uint32_t cout;
    const uint32_t c = wg_carry_scan(run.G, run.P, 0u, scratch, &cout);
    run.apply(c);
#pragma unroll
    for (int i = 0; i < Q; ++i) x[i] = run.s[i];
    total += cout;
  }
  if (VEC && valid == Q) {
#pragma unroll
    for (int i = 0; i < Q; i += 4)
      *reinterpret_cast<uint4*>(po + j0 + i) = make_uint4(x[i], x[i + 1], x[i + 2], x[i + 3]);
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (i < valid) po[j0 + i] = x[i];
  }
  if (ovf && threadIdx.x == 0) ovf[inst] = total;
}

template <int Q>
static int launch_add6_q(uint32_t* out, uint32_t* ovf, const uint32_t* a, const uint32_t* b,
                         int64_t n, int64_t batch, hipStream_t s) {
  const int T = (int)((cdiv(n, Q) + 63) / 64 * 64);
  const bool vec = (n % 4 == 0) && ((uintptr_t)a % 16 == 0) && ((uintptr_t)b % 16 == 0) &&
                   ((uintptr_t)out % 16 == 0);
  if (vec)
    hipLaunchKernelGGL((k_add6<Q, true>), dim3((unsigned)batch), dim3(T), 0, s, out, ovf, a, b,
                       (int)n);
  else
    hipLaunchKernelGGL((k_add6<Q, false>), dim3((unsigned)batch), dim3(T), 0, s, out, ovf, a, b,
                       (int)n);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

int launch_add6(uint32_t* out, uint32_t* ovf, const uint32_t* a, const uint32_t* b, int64_t n,
                int64_t batch, hipStream_t s) {
  // six scans per instance: fewer, fuller threads than for one addition pay
  // (measured: 4.4 TB/s at 4096 limbs with 256 threads, 2.2 with 1024)
  if (n <= kIpbMax) return launch_addsub_ipb<false, 6>(out, ovf, a, b, n, batch, s);
  if (n <= 1024) return launch_add6_q<4>(out, ovf, a, b, n, batch, s);
  if (n <= 2048) return launch_add6_q<8>(out, ovf, a, b, n, batch, s);
  if (n <= 16384) return launch_add6_q<16>(out, ovf, a, b, n, batch, s);
  return BIGINT_EUNSUPPORTED;
}

// Poly: ((a*a + b) * (b*b + b) + a*b) mod B^n.  One work-group per instance
// (instance first + g for work-group g of a launch, workspace slot g): the
// four products mod B^n run one after another on the MFMA-split multiply (a
// single call site, so its code is emitted once) with two n-limb temporaries
// in a global workspace, each followed by its addition on the whole
// work-group.  (A persistent grid looping over instances was 5-16% slower at
// 2^15-2^18 bits: the loop kept loop-invariant values live in registers.)
// Two work-groups per CU need 128 registers (4 waves per SIMD); the 16-strip
// tiles do not fit that, so they keep one.
template <int P>
__global__ __launch_bounds__(512, P == 16 ? 2 : 4) void k_poly(uint32_t* out, const uint32_t* a, const uint32_t* b,
                                              int n, int64_t first, int64_t batch, uint32_t* ws) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ uint32_t scratch[32];
  uint32_t* t1 = ws + (int64_t)blockIdx.x * 2 * n;
  uint32_t* t2 = t1 + n;
  {
    const int64_t inst = first + blockIdx.x;
    if (inst >= batch) return;
    const uint32_t* pa = a + inst * n;
    const uint32_t* pb = b + inst * n;
    uint32_t* po = out + inst * n;
#pragma unroll 1
    for (int op = 0; op < 4; ++op) {
      // products: t1 = a a, t2 = b b, out = t1 t2, t1 = a b
      const uint32_t* x = op == 0 ? pa : (op == 1 ? pb : (op == 2 ? t1 : pa));
      const uint32_t* y = op == 0 ? pa : (op == 1 ? pb : (op == 2 ? t2 : pb));
      uint32_t* dst = op == 0 ? t1 : (op == 1 ? t2 : (op == 2 ? po : t1));
      mfma::wg_mul_mfma<8, P>(dst, nullptr, x, n, y, n, smem, n);
      if (op == 2) continue;
      // sums: t1 += b, t2 += b, out += t1
      uint32_t* acc = op == 3 ? po : dst;
      const uint32_t* add = op == 3 ? t1 : pb;
      auto X = [&](int j) -> uint32_t { return acc[j]; };
      auto Y = [&](int j) -> uint32_t { return add[j]; };
      wg_addsub<16, false>(acc, n, X, Y, 0u, scratch);
    }
  }
}

// Poly for small operands on the one-wave-per-instance multiply: wave g of
// a launch takes instance first + g and workspace slot g (2n limbs), the
// four products mod B^n run on mfma::wave_mul_mfma and the three additions
// on the same wave (64 limbs per step, carries by ballot).
__device__ __forceinline__ void wave_add_into(uint32_t* acc, const uint32_t* add, int n) {
  uint32_t carry = 0u;
  for (int base = 0; base < n; base += 64) {
    const int j = base + lane_id();
    const uint32_t x = j < n ? acc[j] : 0u, y = j < n ? add[j] : 0u;
    const uint32_t r = x + y;
    const WaveCarry w = wave_carry_masks(j < n && r < x, j < n && r == 0xffffffffu);
    const uint32_t c = wave_carry_in(w, carry);
    carry = wave_carry_out(w, carry);
    if (j < n) acc[j] = r + c;
  }
}

template <int P>
__global__ __launch_bounds__(64 * kWaveInst) void k_poly_wave(uint32_t* out, const uint32_t* a,
                                                              const uint32_t* b, int n,
                                                              int64_t first, int64_t batch,
                                                              uint32_t* ws, int wave_lds) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int64_t slot = (int64_t)blockIdx.x * kWaveInst + wave_id();
  const int64_t inst = first + slot;
  if (inst >= batch) return;   // the whole wave
  char* sm = smem + (size_t)wave_id() * wave_lds;
  uint32_t* t1 = ws + slot * 2 * n;
  uint32_t* t2 = t1 + n;
  const uint32_t* pa = a + inst * n;
  const uint32_t* pb = b + inst * n;
  uint32_t* po = out + inst * n;
#pragma unroll 1
  for (int op = 0; op < 4; ++op) {
    // products: t1 = a a, t2 = b b, out = t1 t2, t1 = a b
    const uint32_t* x = op == 0 ? pa : (op == 1 ? pb : (op == 2 ? t1 : pa));
    const uint32_t* y = op == 0 ? pa : (op == 1 ? pb : (op == 2 ? t2 : pb));
    uint32_t* dst = op == 0 ? t1 : (op == 1 ? t2 : (op == 2 ? po : t1));
    mfma::wave_mul_mfma<P>(dst, x, n, y, n, sm, n);
    mfma::wave_sync();
    if (op == 2) continue;
    // sums: t1 += b, t2 += b, out += t1
    wave_add_into(op == 3 ? po : dst, op == 3 ? t1 : pb, n);
    mfma::wave_sync();
  }
}

// instances per Poly wave launch (one workspace slot each): eight times as
// many as stay resident, at most the batch
int poly_wave_chunk(int n, int64_t batch, int P) {
  const size_t lds = (size_t)kWaveInst * mfma::wave_lds_bytes(n, n);
  const void* k = P == 4 ? (const void*)k_poly_wave<4> : (const void*)k_poly_wave<8>;
  int per_cu = 1;
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 64 * kWaveInst, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return (int)std::max<int64_t>(
      1, std::min<int64_t>(batch, 8 * (int64_t)num_cus() * per_cu * kWaveInst));
}

int launch_poly_wave(uint32_t* out, const uint32_t* a, const uint32_t* b, int64_t n, int64_t batch,
                     uint32_t* ws, int chunk, int P, hipStream_t s) {
  const int wl = (int)mfma::wave_lds_bytes((int)n, (int)n);
  const size_t lds = (size_t)kWaveInst * wl;
  if (lds > 163840) return BIGINT_EUNSUPPORTED;
  if (chunk < 1) return BIGINT_EINVAL;
  const void* k = P == 4 ? (const void*)k_poly_wave<4> : (const void*)k_poly_wave<8>;
  BI_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  for (int64_t first = 0; first < batch; first += chunk) {
    const int64_t cnt = std::min<int64_t>(chunk, batch - first);
    const dim3 gd((unsigned)((cnt + kWaveInst - 1) / kWaveInst)), bd(64 * kWaveInst);
    if (P == 4)
      hipLaunchKernelGGL(k_poly_wave<4>, gd, bd, lds, s, out, a, b, (int)n, first,
                         first + cnt, ws, wl);
    else
      hipLaunchKernelGGL(k_poly_wave<8>, gd, bd, lds, s, out, a, b, (int)n, first,
                         first + cnt, ws, wl);
    BI_LAUNCH_CHECK();
  }
  return BIGINT_OK;
}

size_t poly_lds(int n, MfmaCfg cfg) { return mfma::lds_bytes<8>(n, n, cfg.waves, cfg.P) + 256; }

static const void* poly_kernel(int P) {
  return P == 4 ? (const void*)k_poly<4> : (P == 8 ? (const void*)k_poly<8> : (const void*)k_poly<16>);
}

// work-groups per Poly launch (one workspace slot each): eight times as many
// as stay resident together, at most the batch
int poly_chunk(int n, int64_t batch, MfmaCfg cfg) {
  int per_cu = 1;
  const size_t lds = mfma::lds_bytes<8>(n, n, cfg.waves, cfg.P);
  if (hipFuncSetAttribute(poly_kernel(cfg.P), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, poly_kernel(cfg.P), 64 * cfg.waves,
                                                   lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return (int)std::max<int64_t>(1, std::min<int64_t>(batch, 8 * (int64_t)num_cus() * per_cu));
}

int launch_poly(uint32_t* out, const uint32_t* a, const uint32_t* b, int64_t n, int64_t batch,
                uint32_t* ws, int chunk, MfmaCfg cfg, hipStream_t s) {
  const size_t lds = mfma::lds_bytes<8>((int)n, (int)n, cfg.waves, cfg.P);
  if (lds + 256 > 163840) return BIGINT_EUNSUPPORTED;
  if (chunk < 1) return BIGINT_EINVAL;
  BI_HIP(hipFuncSetAttribute(poly_kernel(cfg.P), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds));
  // chunks run one after another on the stream, so a workspace slot is never
  // held by two live work-groups
  for (int64_t first = 0; first < batch; first += chunk) {
    const dim3 gd((unsigned)std::min<int64_t>(chunk, batch - first)), bd(64 * cfg.waves);
    switch (cfg.P) {
      case 4: hipLaunchKernelGGL(k_poly<4>, gd, bd, lds, s, out, a, b, (int)n, first, batch, ws); break;
      case 8: hipLaunchKernelGGL(k_poly<8>, gd, bd, lds, s, out, a, b, (int)n, first, batch, ws); break;
      default: hipLaunchKernelGGL(k_poly<16>, gd, bd, lds, s, out, a, b, (int)n, first, batch, ws); break;
    }
    BI_LAUNCH_CHECK();
  }
  return BIGINT_OK;
}

// ============================================================================
// digit split (diagnostic): out[k] = bits [7k, 7k+7) of a
// ============================================================================
__global__ void k_digits7(uint8_t* out, const uint32_t* a, int n, int D) {
  const int64_t inst = blockIdx.y;
  const uint32_t* pa = a + inst * n;
  uint8_t* po = out + inst * (int64_t)D;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < D; k += gridDim.x * blockDim.x)
    po[k] = (uint8_t)digit7(pa, n, k);
}

int launch_digits7(uint8_t* out, const uint32_t* a, int64_t n, int64_t D, int64_t batch,
                   hipStream_t s) {
  const int blocks = (int)std::min<int64_t>(cdiv(D, 256), 64);
  hipLaunchKernelGGL(k_digits7, dim3(blocks, (unsigned)batch), dim3(256), 0, s, out, a, (int)n,
                     (int)D);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

// ============================================================================
// ragged multiply: the instances ordered largest first form a queue; work-
// group t of a launch multiplies queue entry t.  Work-groups are dispatched in
// index order as earlier ones finish, so a launch runs the queue as a list
// schedule, largest first, without a device-side counter.  (A persistent
// loop pulling entries with an atomic was measured 18% slower at 2^17 bits
// with two work-groups per CU.)  Each launch (a segment of the queue) runs the
// kernel of its leading tile configuration, so it gets that configuration's
// register budget and occupancy; at its end it also takes some instances of
// the next, smaller configurations, so that its last work-groups do not leave
// the chip idle.
// ============================================================================
// Smaller configurations inside a segment (inlined: out of line, the callee's
// own register use raised the kernel's).
template <int DW, int P>
__device__ __forceinline__ void ragged_filler(uint32_t* po, const uint32_t* pa, int na,
                                           const uint32_t* pb, int nb, char* smem) {
  mfma::wg_mul_mfma<DW, P>(po, nullptr, pa, na, pb, nb, smem);
}

template <int DW, int P>
__global__ __launch_bounds__(512) void k_mul_mfma_ragged(uint32_t* out, const int64_t* out_off,
                                                         const uint32_t* a, const int64_t* a_off,
                                                         const uint32_t* b, const int64_t* b_off,
                                                         const QueueItem* queue, int nitems) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int t = blockIdx.x;
  if (t >= nitems) return;
  const int64_t i = __builtin_amdgcn_readfirstlane(queue[t].inst);
  const int p = __builtin_amdgcn_readfirstlane(queue[t].cfg);  // strips per band
  const int na = (int)(a_off[i + 1] - a_off[i]);
  const int nb = (int)(b_off[i + 1] - b_off[i]);
  uint32_t* po = out + out_off[i];
  const uint32_t* pa = a + a_off[i];
  const uint32_t* pb = b + b_off[i];
  if (p == P) {
    mfma::wg_mul_mfma<DW, P>(po, nullptr, pa, na, pb, nb, smem);
  } else if constexpr (P == 16) {
    if (p == 8) ragged_filler<DW, 8>(po, pa, na, pb, nb, smem);
    else ragged_filler<DW, 4>(po, pa, na, pb, nb, smem);
  } else if constexpr (P == 8) {
    ragged_filler<DW, 4>(po, pa, na, pb, nb, smem);
  }
}

// A ragged segment of few instances split like a small uniform batch
// (k_mul_mfma_part): part blockIdx.x of queue entry blockIdx.y, carry words
// at ws[blockIdx.y * wstride + w]; then k_mul_mfma_close_ragged per entry.
template <int DW>
__global__ __launch_bounds__(64 * kSplitWaves) void k_mul_mfma_part_ragged(
    uint32_t* out, const int64_t* out_off, const uint32_t* a, const int64_t* a_off, const uint32_t* b,
    const int64_t* b_off, const QueueItem* queue, int nparts, uint64_t* ws, int wstride) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int t = blockIdx.y;
  const int64_t i = __builtin_amdgcn_readfirstlane(queue[t].inst);
  const int na = (int)(a_off[i + 1] - a_off[i]);
  const int nb = (int)(b_off[i + 1] - b_off[i]);
  mfma::wg_mul_mfma<DW, kSplitP>(out + out_off[i], nullptr, a + a_off[i], na, b + b_off[i], nb, smem, na + nb,
                                 0, (int)blockIdx.x, nparts, ws + (int64_t)t * wstride);
}

template <int DW>
__global__ __launch_bounds__(1024) void k_mul_mfma_close_ragged(uint32_t* out, const int64_t* out_off,
                                                                const int64_t* a_off, const int64_t* b_off,
                                                                const QueueItem* queue, const uint64_t* ws,
                                                                int wstride) {
  __shared__ uint32_t scratch[32];
  const int t = blockIdx.x;
  const int64_t i = __builtin_amdgcn_readfirstlane(queue[t].inst);
  const int na = (int)(a_off[i + 1] - a_off[i]);
  const int nb = (int)(b_off[i + 1] - b_off[i]);
  const mfma::Geo g = mfma::make_geo<DW>(na, nb, na + nb);
  mfma::close_strips<DW>(out + out_off[i], g, ws + (int64_t)t * wstride, 0, scratch);
}

__global__ __launch_bounds__(1024) void k_mul_plain_ragged(uint32_t* out, const int64_t* out_off,
                                                           const uint32_t* a, const int64_t* a_off,
                                                           const uint32_t* b, const int64_t* b_off,
                                                           const QueueItem* queue, int nitems) {
  extern __shared__ uint64_t sm64[];
  const int t = blockIdx.x;
  if (t >= nitems) return;
  const int64_t i = __builtin_amdgcn_readfirstlane(queue[t].inst);
  const int na = (int)(a_off[i + 1] - a_off[i]);
  const int nb = (int)(b_off[i + 1] - b_off[i]);
  wg_mul_plain<kPlainQ, kPlainR>(out + out_off[i], a + a_off[i], na, b + b_off[i], nb, sm64);
}

// ============================================================================
// register-only MFMA rate probe (diagnostic): every wave keeps 8 independent
// accumulators busy with v_mfma_i32_16x16x64_i8, 64 per loop round (so the
// loop's own register moves stay small next to them); no memory traffic.
// toggle != 0 changes every operand bit pattern between rounds (one XOR per
// round), as random digits do; constant operands draw less power.
// ============================================================================
__global__ __launch_bounds__(256) void k_mfma_rate(int32_t* out, int iters, int toggle) {
  const int lane = lane_id();
  v4i a = {lane, lane * 3, lane * 5, lane * 7};
  v4i b = {lane * 11, lane * 13, lane, 1};
  v4i acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = v4i{j, 0, 0, 0};
  const int flip = toggle ? (int)0x9e3779b9 : 0;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[j], 0, 0, 0);
      a ^= flip;
      b ^= flip + r;
    }
  }
  int32_t t = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) t += acc[j].x + acc[j].y + acc[j].z + acc[j].w;
  out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

// ============================================================================
// register-only 32x32+64 -> 64-bit multiply-add rate probe (diagnostic): the
// plain kernel's inner operation (v_mad_u64_u32).  Every lane runs 8
// independent chains acc = a_j * lo32(acc) + acc, 64 per loop round; the
// multiplier changes every step, so nothing can be hoisted.
// ============================================================================
__global__ __launch_bounds__(256) void k_mad_rate(uint64_t* out, int iters) {
  const uint32_t lane = threadIdx.x;
  uint64_t acc[8];
  uint32_t m[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    acc[j] = ((uint64_t)(lane + j) << 32) | (0x9e3779b9u * (lane + 1) + j);
    m[j] = 0x85ebca6bu + 2654435761u * (uint32_t)j + lane;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = (uint64_t)m[j] * (uint32_t)acc[j] + acc[j];
    }
  }
  uint64_t t = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) t ^= acc[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

// number of differing words of two device arrays (the autotuner's identity
// check): one atomic add per wave that saw a difference
__global__ __launch_bounds__(256) void k_count_diff(uint32_t* count, const uint32_t* x,
                                                    const uint32_t* y, size_t n) {
  uint32_t d = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    d += x[i] != y[i];
  for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
  if (lane_id() == 0 && d) atomicAdd(count, d);
}

int launch_count_diff(uint32_t* count, const uint32_t* x, const uint32_t* y, size_t n, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<size_t>(std::max<size_t>(cdiv((int64_t)n, 256), 1), 8192);
  hipLaunchKernelGGL(k_count_diff, dim3(blocks), dim3(256), 0, s, count, x, y, n);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

int launch_mad_rate(uint64_t* out, int blocks, int iters, hipStream_t s) {
  hipLaunchKernelGGL(k_mad_rate, dim3(blocks), dim3(256), 0, s, out, iters);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

// The same probe on v_mfma_i32_32x32x32_i8 (32,768 multiply-accumulates per
// instruction, twice the 16x16x64 tile's for the same 16 operand bytes per
// lane): 4 independent 32x32 accumulators per wave, 32 MFMAs per loop
// round (the same multiply-accumulates per round as the 16x16x64 probe).
typedef int v16i __attribute__((ext_vector_type(16)));
__global__ __launch_bounds__(256) void k_mfma_rate32(int32_t* out, int iters, int toggle) {
  const int lane = lane_id();
  v4i a = {lane, lane * 3, lane * 5, lane * 7};
  v4i b = {lane * 11, lane * 13, lane, 1};
  v16i acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[j][e] = e == 0 ? j : 0;
  }
  const int flip = (toggle & 1) ? (int)0x9e3779b9 : 0;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[j], 0, 0, 0);
      a ^= flip;
      b ^= flip + r;
    }
  }
  int32_t t = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
#pragma unroll
    for (int e = 0; e < 16; ++e) t += acc[j][e];
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

int launch_mfma_rate(int32_t* out, int blocks, int iters, int toggle, hipStream_t s) {
  if (toggle & 2)
    hipLaunchKernelGGL(k_mfma_rate32, dim3(blocks), dim3(256), 0, s, out, iters, toggle);
  else
    hipLaunchKernelGGL(k_mfma_rate, dim3(blocks), dim3(256), 0, s, out, iters, toggle);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}


template <int DW, int P>
static const void* ragged_kernel_p() {
  return (const void*)k_mul_mfma_ragged<DW, P>;
}

static const void* ragged_kernel(int cfg_id) {
  switch (cfg_id) {
    case 0: return ragged_kernel_p<7, 4>();
    case 1: return ragged_kernel_p<7, 8>();
    case 2: return ragged_kernel_p<7, 16>();
    case 3: return ragged_kernel_p<8, 4>();
    case 4: return ragged_kernel_p<8, 8>();
    case 5: return ragged_kernel_p<8, 16>();
    default: return nullptr;
  }
}

int ragged_slots(int cfg_id, int waves, size_t lds) {
  const void* k = ragged_kernel(cfg_id);
  if (!k || lds > 163840) return 0;
  int per_cu = 1;
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 64 * waves, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return num_cus() * per_cu;
}

template <int DW, int P>
static void launch_ragged_class(const RaggedClass& c, uint32_t* out, const int64_t* out_off,
                                const uint32_t* a, const int64_t* a_off, const uint32_t* b,
                                const int64_t* b_off, const QueueItem* queue, hipStream_t s) {
  hipLaunchKernelGGL((k_mul_mfma_ragged<DW, P>), dim3(c.count), dim3(64 * c.waves), c.lds, s, out,
                     out_off, a, a_off, b, b_off, queue + c.first, c.count);
}

template <int DW>
static int launch_ragged_split(const RaggedClass& c, uint32_t* out, const int64_t* out_off, const uint32_t* a,
                               const int64_t* a_off, const uint32_t* b, const int64_t* b_off,
                               const QueueItem* queue, uint64_t* ws, hipStream_t s) {
  BI_HIP(hipFuncSetAttribute((const void*)k_mul_mfma_part_ragged<DW>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.split_lds));
  hipLaunchKernelGGL(k_mul_mfma_part_ragged<DW>, dim3((unsigned)c.parts, (unsigned)c.count),
                     dim3(64 * kSplitWaves), c.split_lds, s, out, out_off, a, a_off, b, b_off,
                     queue + c.first, c.parts, ws + c.ws_off, c.wstride);
  BI_LAUNCH_CHECK();
  const unsigned threads = (unsigned)std::min(1024, (c.wstride + 63) / 64 * 64);
  hipLaunchKernelGGL(k_mul_mfma_close_ragged<DW>, dim3((unsigned)c.count), dim3(threads), 0, s, out,
                     out_off, a_off, b_off, queue + c.first, ws + c.ws_off, c.wstride);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

int launch_mul_ragged(uint32_t* out, const int64_t* out_off, const uint32_t* a,
                      const int64_t* a_off, const uint32_t* b, const int64_t* b_off,
                      const QueueItem* queue, const RaggedClass* cls, int ncls, void* ws_v,
                      hipStream_t s) {
  uint64_t* ws = reinterpret_cast<uint64_t*>(ws_v);
  for (int k = 0; k < ncls; ++k) {
    const RaggedClass& c = cls[k];
    if (c.parts > 1) {
      if (!ws || c.split_lds > 163840) return BIGINT_EINVAL;
      const int rc = c.cfg >= 3 ? launch_ragged_split<8>(c, out, out_off, a, a_off, b, b_off, queue, ws, s)
                                : launch_ragged_split<7>(c, out, out_off, a, a_off, b, b_off, queue, ws, s);
      if (rc != BIGINT_OK) return rc;
      continue;
    }
    const void* kern = ragged_kernel(c.cfg);
    if (!kern || c.lds > 163840) return BIGINT_EUNSUPPORTED;
    if (c.count < 1) continue;
    BI_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds));
    switch (c.cfg) {
      case 0: launch_ragged_class<7, 4>(c, out, out_off, a, a_off, b, b_off, queue, s); break;
      case 1: launch_ragged_class<7, 8>(c, out, out_off, a, a_off, b, b_off, queue, s); break;
      case 2: launch_ragged_class<7, 16>(c, out, out_off, a, a_off, b, b_off, queue, s); break;
      case 3: launch_ragged_class<8, 4>(c, out, out_off, a, a_off, b, b_off, queue, s); break;
      case 4: launch_ragged_class<8, 8>(c, out, out_off, a, a_off, b, b_off, queue, s); break;
      default: launch_ragged_class<8, 16>(c, out, out_off, a, a_off, b, b_off, queue, s); break;
    }
    BI_LAUNCH_CHECK();
  }
  return BIGINT_OK;
}

int launch_mul_plain_ragged(uint32_t* out, const int64_t* out_off, const uint32_t* a,
                            const int64_t* a_off, const uint32_t* b, const int64_t* b_off,
                            const QueueItem* queue, int64_t nitems, size_t lds, hipStream_t s) {
  BI_HIP(hipFuncSetAttribute((const void*)k_mul_plain_ragged,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_mul_plain_ragged, dim3((unsigned)nitems), dim3(1024), lds, s, out, out_off,
                     a, a_off, b, b_off, queue, (int)nitems);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

}  // namespace bi
