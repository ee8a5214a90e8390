// kernels_div.hip -- division kernels: one work-group per division, pulling
// instances from a queue (largest first) until the queue is empty.
#include <algorithm>

#include "internal.hpp"
#include "dev_divmod.hpp"

namespace bi {

// threads per division work-group
constexpr int kDivThreads = 512;

__global__ void k_zero_u32_div(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Uniform batches pass null offsets and the limb counts nu / nv; ragged
// batches pass prefix offsets.  queue == nullptr means instance t is item t.
// h_inv >= 0 selects the shifted-inverse diagnostic: q[i] = floor(B^h_inv / v).
__global__ __launch_bounds__(kDivThreads, 4) void k_divmod(uint32_t* q, const int64_t* q_off, uint32_t* r,
                                                const int64_t* r_off, int32_t* status,
                                                const uint32_t* u, const int64_t* u_off, int nu,
                                                const uint32_t* v, const int64_t* v_off, int nv,
                                                const int32_t* queue, int nitems, uint32_t* counter,
                                                uint32_t* ws, int cap_u, int cap_v, int h_inv,
                                                int32_t* adjust) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ div::Shared sh;
  __shared__ int item;
  uint32_t* myws = ws + (size_t)blockIdx.x * div::div_ws_limbs(cap_u, cap_v);
  const div::Bufs bf = div::carve_bufs(myws, cap_u, cap_v);
  for (;;) {
    if (threadIdx.x == 0) item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(item);
    __syncthreads();
    if (t >= nitems) break;
    const int64_t i = queue ? (int64_t)__builtin_amdgcn_readfirstlane(queue[t]) : (int64_t)t;
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
    int adj = 0;
    const int st = div::wg_divmod(q + qo, lq, r ? r + ro : nullptr, lr, u ? u + uo : nullptr, lu,
                                  v + vo, lv, bf, &sh, smem, h_inv >= 0, h_inv, &adj);
    if (threadIdx.x == 0) {
      if (status) status[i] = st;
      if (adjust) adjust[i] = adj;
    }
    __syncthreads();
  }
}

size_t div_ws_bytes(int cap_u, int cap_v, int grid) {
  return (size_t)grid * div::div_ws_limbs(cap_u, cap_v) * 4 + 256;
}

size_t div_lds_bytes(int cap_u, int cap_v) {
  // the largest product of a division has two factors of at most cap_u + 8 limbs
  const int m = cap_u + 8;
  (void)cap_v;
  return mfma::lds_bytes<div::kDW>(m, m, kDivThreads / 64, div::kP);
}

// Work-groups that fit one CU: the kernel is built for 4 waves per SIMD (16
// per CU), so that many waves and then the LDS decide.
int div_groups_per_cu(int cap_u, int cap_v) {
  const size_t per = div_lds_bytes(cap_u, cap_v) + sizeof(div::Shared) + 64;
  const int by_waves = 16 / (kDivThreads / 64);
  return std::max(1, std::min<int>(by_waves, (int)(163840 / per)));
}

int launch_divmod(uint32_t* q, const int64_t* q_off, uint32_t* r, const int64_t* r_off,
                  int32_t* status, const uint32_t* u, const int64_t* u_off, int nu,
                  const uint32_t* v, const int64_t* v_off, int nv, const int32_t* queue,
                  int64_t nitems, void* ws, int cap_u, int cap_v, int grid, int h_inv,
                  int32_t* adjust, hipStream_t s) {
  uint32_t* counter = reinterpret_cast<uint32_t*>(ws);
  uint32_t* bufs = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(ws) + 256);
  const size_t lds = div_lds_bytes(cap_u, cap_v);
  if (lds > 163840 - sizeof(div::Shared) - 64) return BIGINT_EUNSUPPORTED;
  hipLaunchKernelGGL(k_zero_u32_div, dim3(1), dim3(64), 0, s, counter, 1);
  BI_LAUNCH_CHECK();
  BI_HIP(hipFuncSetAttribute((const void*)k_divmod, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds));
  hipLaunchKernelGGL(k_divmod, dim3(grid), dim3(kDivThreads), lds, s, q, q_off, r, r_off, status, u, u_off,
                     nu, v, v_off, nv, queue, (int)nitems, counter, bufs, cap_u, cap_v, h_inv,
                     adjust);
  BI_LAUNCH_CHECK();
  return BIGINT_OK;
}

}  // namespace bi
