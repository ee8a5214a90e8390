// kernels_div.hip -- division kernels: one work-group per division, the
// divisions taken in queue order (largest first).
#include <algorithm>
#include <mutex>

#include "internal.hpp"
#include "dev_divmod.hpp"

namespace bi {

// threads per division work-group: at most kDivThreads (the register budget
// is that of 4 waves per SIMD).  A division is mostly a chain of short
// latency-bound passes, so smaller dividends run on fewer threads and more
// divisions share a CU: 64 threads up to 1448 dividend limbs, 128 up to
// 2896, 256 up to 5792 (measured on uniform batches of 2^13..2^18-bit
// dividends: 6.9x faster at 2^13 bits than with 512 threads, the same at 2^18).
constexpr int kDivThreads = 512;
constexpr int kDivT64 = 1448, kDivT128 = 2896, kDivT256 = 5792;

int div_threads(int cap_u) {
  return cap_u <= kDivT64 ? 64 : (cap_u <= kDivT128 ? 128 : (cap_u <= kDivT256 ? 256 : kDivThreads));
}

// Uniform batches pass null offsets and the limb counts nu / nv; ragged
// batches pass prefix offsets.  queue == nullptr means instance t is item t.
// Work-group g of a launch takes item first + g and workspace slot g.  Work-
// groups are dispatched in index order, so the items run as a list schedule
// in queue order.  (A persistent loop pulling items with an atomic was
// measured 11% slower on 512 ragged divisions: the loop made the compiler
// keep loop-invariant values live across the whole division.)
// h_inv >= 0 selects the shifted-inverse diagnostic: q[i] = floor(B^h_inv / v).
// adjust (nullable): 4 int64 per instance, the division's counters (Newton
// steps, fix-up unit steps, quotient corrections, MFMA multiply-accumulates).
__global__ __launch_bounds__(kDivThreads, 4) void k_divmod(uint32_t* q, const int64_t* q_off, uint32_t* r,
                                                const int64_t* r_off, int32_t* status,
                                                const uint32_t* u, const int64_t* u_off, int nu,
                                                const uint32_t* v, const int64_t* v_off, int nv,
                                                const int32_t* queue, int64_t first, int64_t nitems,
                                                uint32_t* ws, int cap_u, int cap_v, int h_inv,
                                                int64_t* adjust) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ div::Shared sh;
  const int64_t t = first + blockIdx.x;
  if (t >= nitems) return;
  uint32_t* myws = ws + (size_t)blockIdx.x * div::div_ws_limbs(cap_u, cap_v);
  const div::Bufs bf = div::carve_bufs(myws, cap_u, cap_v);
  const int64_t i = queue ? (int64_t)__builtin_amdgcn_readfirstlane(queue[t]) : t;
  int64_t uo, vo, qo, ro;
  int lu, lv, lq, lr;
  if (u_off) {
    uo = u_off[i]; lu = (int)(u_off[i + 1] - uo);
    vo = v_off[i]; lv = (int)(v_off[i + 1] - vo);
    qo = q_off[i]; lq = (int)(q_off[i + 1] - qo);
    ro = r_off ? r_off[i] : 0; lr = r_off ? (int)(r_off[i + 1] - ro) : 0;
  } else {
    lu = nu; lv = nv;
    uo = i * (int64_t)nu; vo = i * (int64_t)nv;
    lq = h_inv >= 0 ? h_inv + 1 : nu; qo = i * (int64_t)lq;
    lr = nv; ro = i * (int64_t)nv;
  }
  int64_t cnt[4] = {0, 0, 0, 0};
  const int st = div::wg_divmod(q + qo, lq, r ? r + ro : nullptr, lr, u ? u + uo : nullptr, lu,
                                v + vo, lv, bf, &sh, smem, h_inv >= 0, h_inv, cnt);
  if (threadIdx.x == 0) {
    if (status) status[i] = st;
    if (adjust) {
#pragma unroll
      for (int j = 0; j < 4; ++j) adjust[4 * i + j] = cnt[j];
    }
  }
}

size_t div_ws_bytes(int cap_u, int cap_v, int slots) {
  return (size_t)slots * div::div_ws_limbs(cap_u, cap_v) * 4;
}

size_t div_lds_bytes(int cap_u, int cap_v) {
  // the largest product of a division has two factors of at most cap_u + 8 limbs
  const int m = cap_u + 8;
  (void)cap_v;
  // (and at least what the small-operand product and the one-wave steps need)
  return std::max<size_t>(mfma::lds_bytes<div::kDW>(m, m, div_threads(cap_u) / 64, div::kP),
                          std::max(div::kSmallMulLds, div::kEarlyLds));
}

// Work-groups that fit one CU: the kernel is built for 4 waves per SIMD (16
// per CU), so that many waves (over the work-group's) and then the LDS decide.
int div_groups_per_cu(int cap_u, int cap_v) {
  const size_t per = div_lds_bytes(cap_u, cap_v) + sizeof(div::Shared) + 64;
  const int by_waves = 16 / (div_threads(cap_u) / 64);
  return std::max(1, std::min<int>(by_waves, (int)(163840 / per)));
}

int div_chunk(int cap_u, int cap_v, int64_t batch) {
  const int64_t resident = (int64_t)num_cus() * div_groups_per_cu(cap_u, cap_v);
  return (int)std::max<int64_t>(1, std::min<int64_t>(batch, 8 * resident));
}

// ---- workspace of the allocation-free division (bigint_divmod_noalloc) ----------
// A file-scope device array, one copy per GPU, held until the process ends.
// Every call on a GPU shares that GPU's copy (calls that overlap on one GPU
// race); the division needs none of it cleared.  In host code the array's
// name is only a stand-in: its device address comes from
// hipGetSymbolAddress, looked up once per device and kept.
constexpr size_t kDivScratchBytes = (size_t)128 << 20;
__device__ __align__(256) uint8_t scratch[kDivScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int div_scratch(void** ptr, size_t* bytes) {
  int dev = 0;
  BI_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return BIGINT_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    BI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return BIGINT_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  *bytes = kDivScratchBytes;
  return BIGINT_OK;
}

int launch_divmod(uint32_t* q, const int64_t* q_off, uint32_t* r, const int64_t* r_off,
                  int32_t* status, const uint32_t* u, const int64_t* u_off, int nu,
                  const uint32_t* v, const int64_t* v_off, int nv, const int32_t* queue,
                  int64_t nitems, void* ws, int cap_u, int cap_v, int chunk, int h_inv,
                  int64_t* adjust, hipStream_t s) {
  const size_t lds = div_lds_bytes(cap_u, cap_v);
  if (lds > 163840 - sizeof(div::Shared) - 64) return BIGINT_EUNSUPPORTED;
  if (chunk < 1) return BIGINT_EINVAL;
  BI_HIP(hipFuncSetAttribute((const void*)k_divmod, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds));
  // chunks run one after another on the stream, so a workspace slot is never
  // held by two live work-groups
  for (int64_t first = 0; first < nitems; first += chunk) {
    const int64_t g = std::min<int64_t>(chunk, nitems - first);
    hipLaunchKernelGGL(k_divmod, dim3((unsigned)g), dim3(div_threads(cap_u)), lds, s, q, q_off, r, r_off,
                       status, u, u_off, nu, v, v_off, nv, queue, first, nitems,
                       reinterpret_cast<uint32_t*>(ws), cap_u, cap_v, h_inv, adjust);
    BI_LAUNCH_CHECK();
  }
  return BIGINT_OK;
}

}  // namespace bi
