// internal.hpp -- host-side launchers shared by the C-ABI translation units.
#pragma once

#include "common.hpp"

namespace bi {

// tile configuration of the MFMA multiply
struct MfmaCfg {
  int P;       // strips per wave band (4, 8, 16; 8, 16, 32 with 32x32 tiles)
  int waves;   // waves per work-group (4, 8); 1: one wave per instance, 4 instances
               // per work-group (8-bit digits, na + nb <= 4096 limbs)
  int dw;      // digit width: 7 (plain 7-bit digits) or 8 (offset 8-bit digits)
  int tile = 16;  // MFMA tile: 16 (v_mfma_i32_16x16x64_i8) or 32 (v_mfma_i32_32x32x32_i8;
                  // 8-bit digits, P = 8 or 16 strips per band)
};

// index of a tile configuration in the ragged kernel's dispatch
inline int ragged_cfg_id(MfmaCfg c) {
  return (c.dw == 8 ? 3 : 0) + (c.P == 4 ? 0 : (c.P == 8 ? 1 : 2));
}

MfmaCfg default_mfma_cfg(int na, int nb);
MfmaCfg current_mfma_cfg(int na, int nb);  // thread override or default
int num_cus();

int launch_addsub(bool sub, uint32_t* out, uint32_t* cout, const uint32_t* a, const uint32_t* b,
                  int64_t n, int64_t batch, hipStream_t s);
int launch_mul_plain(uint32_t* out, const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb,
                     int64_t batch, hipStream_t s);
// products (mod B^nout) of fewer instances than CUs, bands split over work-groups
int mul_mfma_split_parts(int na, int nb, int nout, int64_t batch, int dw, int* wstride);
int launch_mul_mfma_split(uint32_t* out, const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb,
                          int nout, int64_t batch, int dw, int nparts, uint64_t* ws, int wstride,
                          hipStream_t s);
int launch_mul_mfma(uint32_t* out, int32_t* coef, const uint32_t* a, int64_t na,
                    const uint32_t* b, int64_t nb, int64_t batch, MfmaCfg cfg, hipStream_t s,
                    int nout = -1);
size_t kara_ws_bytes(int n, int64_t batch);
int launch_mul_kara(uint32_t* out, const uint32_t* a, const uint32_t* b, int64_t n, int64_t batch,
                    void* ws, MfmaCfg cfg, hipStream_t s);
int launch_add6(uint32_t* out, uint32_t* ovf, const uint32_t* a, const uint32_t* b, int64_t n,
                int64_t batch, hipStream_t s);
size_t poly_lds(int n, MfmaCfg cfg);
int poly_chunk(int n, int64_t batch, MfmaCfg cfg);  // work-groups (workspace slots) per launch
// Poly on the one-wave-per-instance multiply (8-bit digits, P = 4 or 8)
int poly_wave_chunk(int n, int64_t batch, int P);   // instances (workspace slots) per launch
int launch_poly_wave(uint32_t* out, const uint32_t* a, const uint32_t* b, int64_t n, int64_t batch,
                     uint32_t* ws, int chunk, int P, hipStream_t s);
int launch_poly(uint32_t* out, const uint32_t* a, const uint32_t* b, int64_t n, int64_t batch,
                uint32_t* ws, int chunk, MfmaCfg cfg, hipStream_t s);
int launch_digits7(uint8_t* out, const uint32_t* a, int64_t n, int64_t D, int64_t batch,
                   hipStream_t s);

size_t mfma_lds(int na, int nb, MfmaCfg cfg);
bool mfma_wave_fits(int64_t na, int64_t nb);   // the one-wave-per-instance kernel takes it
size_t plain_lds(int na, int nb);

// ---- ragged (persistent, queue-fed) -------------------------------------------
// One queue entry per instance, largest first, one work-group each.  MFMA
// plans cut the queue into segments, one launch each (see RaggedClass); the
// plain plan is one launch.
struct QueueItem {
  int32_t inst;
  int32_t cfg;   // MFMA: strips per band (4, 8, 16) of the instance; plain: 0
};

// One launch of a ragged MFMA plan: queue entries [first, first + count), one
// work-group each, run by the kernel of the segment's leading tile
// configuration (digit width and strips per band of cfg), which also takes
// entries of the same digit width with fewer strips per band.
struct RaggedClass {
  int cfg;        // ragged_cfg_id of the leading configuration
  int waves;      // waves per work-group
  int first;      // first queue entry of the segment
  int count;      // entries
  size_t lds;     // dynamic LDS bytes (largest instance of the segment)
  // parts > 1: every instance's bands split over `parts` work-groups (few
  // instances; the split configuration, 4 strips per band and 4 waves),
  // carry words at workspace words [ws_off + t * wstride ..) for entry t
  int parts = 1;
  int64_t ws_off = 0;
  int wstride = 0;
  size_t split_lds = 0;
};
// strips and part-kernel LDS of one instance of a split ragged segment
void ragged_split_geo(int na, int nb, int dw, int* strips, size_t* lds);

// work-groups of the segment kernel resident on the device at once (0: the
// configuration or LDS size is not supported)
int ragged_slots(int cfg_id, int waves, size_t lds);
int launch_mul_ragged(uint32_t* out, const int64_t* out_off, const uint32_t* a,
                      const int64_t* a_off, const uint32_t* b, const int64_t* b_off,
                      const QueueItem* queue, const RaggedClass* cls, int ncls, void* ws,
                      hipStream_t s);
int launch_mul_plain_ragged(uint32_t* out, const int64_t* out_off, const uint32_t* a,
                            const int64_t* a_off, const uint32_t* b, const int64_t* b_off,
                            const QueueItem* queue, int64_t nitems, size_t lds, hipStream_t s);

int launch_mfma_rate(int32_t* out, int blocks, int iters, int toggle, hipStream_t s);
// *count += the number of indices i < n with x[i] != y[i] (count is device memory)
int launch_count_diff(uint32_t* count, const uint32_t* x, const uint32_t* y, size_t n, hipStream_t s);
int launch_mad_rate(uint64_t* out, int blocks, int iters, hipStream_t s);

// ---- division -------------------------------------------------------------------
// A division launch runs at most `chunk` work-groups at once (one workspace
// slot each, div_ws_bytes(cap_u, cap_v, chunk) bytes in all); larger batches
// go in consecutive launches.
size_t div_ws_bytes(int cap_u, int cap_v, int slots);
size_t div_lds_bytes(int cap_u, int cap_v);
int div_groups_per_cu(int cap_u, int cap_v);
int div_threads(int cap_u);   // threads per division work-group
int div_chunk(int cap_u, int cap_v, int64_t batch);
// The allocation-free division's device workspace on the current device:
// its address (from hipGetSymbolAddress, once per device) and size.
int div_scratch(void** ptr, size_t* bytes);
int launch_divmod(uint32_t* q, const int64_t* q_off, uint32_t* r, const int64_t* r_off,
                  int32_t* status, const uint32_t* u, const int64_t* u_off, int nu,
                  const uint32_t* v, const int64_t* v_off, int nv, const int32_t* queue,
                  int64_t nitems, void* ws, int cap_u, int cap_v, int chunk, int h_inv,
                  int64_t* adjust, hipStream_t s);

}  // namespace bi
