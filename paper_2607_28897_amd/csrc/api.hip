// api.hip -- the C-ABI entry points: argument checks, dispatch, plans.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <queue>
#include <string>
#include <vector>

#include "internal.hpp"

namespace bi {

static thread_local int t_last_hip = 0;
void set_hip_error(hipError_t e) { t_last_hip = (int)e; }

static thread_local int t_cfg_P = 0, t_cfg_waves = 0, t_cfg_dw = 0, t_cfg_tile = 0;

// BIGINT_DEBUG (set, and not "0"): one line on stderr per configuration the
// library picks (multiply calls, plan segments, division launches)
static bool debug_on() {
  static const bool on = [] {
    const char* e = std::getenv("BIGINT_DEBUG");
    return e && *e && std::strcmp(e, "0") != 0;
  }();
  return on;
}
#define BI_DEBUG(...)                                  \
  do {                                                 \
    if (debug_on()) std::fprintf(stderr, __VA_ARGS__); \
  } while (0)

// Tile choice per size bin.  The built-in table is what bigint_autotune
// picked on an MI355X; a table loaded with bigint_autotune_load (or produced
// by bigint_autotune) replaces it.
struct TuneEntry {
  int max_limbs;  // bin upper bound (operand limbs)
  int P, waves, dw;
  int tile = 16;  // MFMA tile (16 or 32)
};
static std::mutex g_tune_mu;
// (waves 1: one wave per instance, four instances per work-group).  8
// strips on 8 waves run up to 8,676 limbs, the largest size whose LDS fits
// two such work-groups on a CU; above it, with one work-group per CU either
// way, 16 strips win (1024 products of 9,000 / 10,000 limbs: 0.599 / 0.615
// of the int8 peak against 0.583 / 0.600).
static const std::vector<TuneEntry> kBuiltinTune = {
    {512, 4, 1, 8}, {1448, 8, 1, 8}, {2896, 8, 4, 8}, {5792, 8, 8, 8}, {8676, 8, 8, 8},
    {BIGINT_MFMA_MAX_LIMBS, 16, 8, 8}};
static std::vector<TuneEntry> g_tune = kBuiltinTune;

static int load_tune_file(const char* path);

// A table named by the environment variable BIGINT_TUNE_CACHE is loaded once,
// before the first lookup and before any table a caller loads or tunes (so
// those replace it); a file that does not parse leaves the built-in table.
static void tune_env_once() {
  static std::once_flag once;
  std::call_once(once, [] {
    const char* path = std::getenv("BIGINT_TUNE_CACHE");
    if (path && *path) (void)load_tune_file(path);
  });
}

// The tuned configuration for this size; when its LDS does not fit (7-bit
// digits near the top of the range) the same tiles with 8-bit digits, which
// need 8/7 fewer bytes per operand.
MfmaCfg default_mfma_cfg(int na, int nb) {
  tune_env_once();
  const int n = std::max(na, nb);
  MfmaCfg c{16, 8, 8};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& e : g_tune)
      if (n <= e.max_limbs) {
        c = MfmaCfg{e.P, e.waves, e.dw, e.tile};
        break;
      }
  }
  if (c.dw == 7 && mfma_lds(na, nb, c) > 163840) c.dw = 8;
  return c;
}

// 32x32 tiles need 8-bit digits, whole tiles per band (8 or 16 strips), a
// work-group of their own and room in LDS for their wider zero padding
// (near 18,432 limbs with 8 waves it does not fit): otherwise 16x16 tiles
static MfmaCfg valid_tile(MfmaCfg c, int na, int nb) {
  if (c.tile == 32 && (c.dw != 8 || (c.P != 8 && c.P != 16 && c.P != 32) || c.waves == 1 ||
                       mfma_lds(na, nb, c) > 163840))
    c.tile = 16;
  if (c.tile == 16 && c.P == 32) c.P = 16;   // 16x16 bands hold at most 16 strips
  return c;
}

// Ragged plans run one instance per work-group: a one-wave-per-instance
// entry of the table becomes 4 waves there.
static MfmaCfg ragged_mfma_cfg(int na, int nb) {
  MfmaCfg c = default_mfma_cfg(na, nb);
  if (c.waves == 1) c.waves = 4;
  c.tile = 16;   // the ragged kernels run 16x16 tiles
  return c;
}

MfmaCfg current_mfma_cfg(int na, int nb) {
  MfmaCfg c = default_mfma_cfg(na, nb);
  if (t_cfg_P) c.P = t_cfg_P;
  if (t_cfg_waves) c.waves = t_cfg_waves;
  if (t_cfg_dw) c.dw = t_cfg_dw;
  if (t_cfg_tile) c.tile = t_cfg_tile;
  return valid_tile(c, na, nb);
}

// One wave per instance pays only once the batch keeps every CU busy with
// several instances, since the latency of one instance on one wave grows
// with na*nb.  Measured crossovers on MI355X (128..1024 limbs), in instances:
// about na*nb/64 for full products (256 at 128 limbs, 1024 at 256, 4096 at
// 512, 16384 at 1024), n*n/256 for products mod B^n (half the strips), and
// n*n/16 for Poly (its four products and three additions per wave).  Smaller
// uniform batches run 4 waves per instance: full products with the table's
// strips per band, products mod B^n and Poly with 4 strips per band, so that
// their fewer bands still reach all four waves.  At 64 pairs of 1024 limbs
// that is 2.5x faster.  Settings of bigint_set_mfma_config are kept.
constexpr int kWaveFull = 64, kWaveLow = 256, kWavePoly = 16;

static bool wave_batch(int64_t na, int64_t nb, int64_t batch, int per) {
  return batch * per >= na * nb;
}

static MfmaCfg uniform_mfma_cfg(int na, int nb, int64_t batch, bool low) {
  MfmaCfg c = current_mfma_cfg(na, nb);
  bool one = false;
  if (c.waves == 1 && t_cfg_waves == 0 && !wave_batch(na, nb, batch, low ? kWaveLow : kWaveFull)) {
    c.waves = 4;
    one = true;
    if (low && t_cfg_P == 0) c.P = 4;
  }
  // Fewer instances than CUs: every work-group has a CU to itself, and 8
  // waves (two per SIMD) hide more MFMA and LDS latency than 4.  Measured
  // (call times through the Python binding): full products of 64 x 1024 limbs
  // 26.3 -> 22.6 us (4 strips per band), 64 x 2048 limbs 39.7 -> 34.4 us (the
  // table's 8 strips); products mod B^n of 64 x 2048 limbs 31.2 -> 27.0 us
  // (4 strips per band; 8 strips gain nothing there).
  if (c.waves == 4 && t_cfg_waves == 0 && batch < num_cus()) {
    MfmaCfg w = c;
    w.waves = 8;
    if ((one || low) && t_cfg_P == 0) w.P = 4;
    if (mfma_lds(na, nb, w) <= 163840) c = w;
  }
  return valid_tile(c, na, nb);
}

// CU count of the device current at the first call (one initialisation,
// thread-safe; every device the library drives is the same part)
int num_cus() {
  static const int n = [] {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cu <= 0)
      cu = 256;
    return cu;
  }();
  return n;
}

// byte ranges [p, p+n) overlap?
static bool overlap(const void* p, size_t n, const void* q, size_t m) {
  if (!p || !q || n == 0 || m == 0) return false;
  const uintptr_t a = (uintptr_t)p, b = (uintptr_t)q;
  return a < b + m && b < a + n;
}

}  // namespace bi

using namespace bi;

extern "C" {

int bigint_version(void) { return 10000; }

const char* bigint_strerror(int code) {
  switch (code) {
    case BIGINT_OK: return "success";
    case BIGINT_EINVAL: return "invalid argument";
    case BIGINT_ENOMEM: return "out of memory";
    case BIGINT_EHIP: return "HIP runtime error";
    case BIGINT_EUNSUPPORTED: return "size outside the supported range";
    default: return "unknown status code";
  }
}

int bigint_last_hip_error(void) { return t_last_hip; }

int bigint_set_mfma_config(int strips_per_band, int waves, int digit_bits) {
  if (strips_per_band != 0 && strips_per_band != 4 && strips_per_band != 8 &&
      strips_per_band != 16 && strips_per_band != 32)
    return BIGINT_EINVAL;
  if (waves != 0 && waves != 1 && waves != 4 && waves != 8) return BIGINT_EINVAL;
  if (digit_bits != 0 && digit_bits != 7 && digit_bits != 8) return BIGINT_EINVAL;
  t_cfg_P = strips_per_band;
  t_cfg_waves = waves;
  t_cfg_dw = digit_bits;
  return BIGINT_OK;
}

int bigint_set_mfma_tile(int tile) {
  if (tile != 0 && tile != 16 && tile != 32) return BIGINT_EINVAL;
  t_cfg_tile = tile;
  return BIGINT_OK;
}

int bigint_mfma_tile(int64_t na, int64_t nb) {
  if (na <= 0 || nb <= 0) return BIGINT_EINVAL;
  if (na > BIGINT_MFMA_MAX_LIMBS || nb > BIGINT_MFMA_MAX_LIMBS) return BIGINT_EUNSUPPORTED;
  return current_mfma_cfg((int)na, (int)nb).tile;
}

int bigint_mfma_config(int64_t na, int64_t nb, int* strips_per_band, int* waves, int* digit_bits) {
  if (na <= 0 || nb <= 0 || !strips_per_band || !waves || !digit_bits) return BIGINT_EINVAL;
  if (na > BIGINT_MFMA_MAX_LIMBS || nb > BIGINT_MFMA_MAX_LIMBS) return BIGINT_EUNSUPPORTED;
  const MfmaCfg c = current_mfma_cfg((int)na, (int)nb);
  *strips_per_band = c.P;
  *waves = c.waves;
  *digit_bits = c.dw;
  return mfma_lds((int)na, (int)nb, c) <= 163840 ? BIGINT_OK : BIGINT_EUNSUPPORTED;
}

static int addsub_common(bool sub, uint32_t* out, uint32_t* cout, const uint32_t* a,
                         const uint32_t* b, int64_t n, int64_t batch, void* stream) {
  if (!out || !a || !b || n <= 0 || batch < 0) return BIGINT_EINVAL;
  if (n > 65536) return BIGINT_EUNSUPPORTED;
  if (batch > 0x7fffffff) return BIGINT_EUNSUPPORTED;
  const size_t bytes = (size_t)n * (size_t)batch * 4;
  // in place is allowed only exactly
  if (out != a && overlap(out, bytes, a, bytes)) return BIGINT_EINVAL;
  if (out != b && overlap(out, bytes, b, bytes)) return BIGINT_EINVAL;
  if (cout) {
    const size_t cb = (size_t)batch * 4;
    if (overlap(cout, cb, out, bytes) || overlap(cout, cb, a, bytes) || overlap(cout, cb, b, bytes))
      return BIGINT_EINVAL;
  }
  if (batch == 0) return BIGINT_OK;
  return launch_addsub(sub, out, cout, a, b, n, batch, (hipStream_t)stream);
}

int bigint_add(uint32_t* out, uint32_t* carry_out, const uint32_t* a, const uint32_t* b, int64_t n,
               int64_t batch, void* stream) {
  return addsub_common(false, out, carry_out, a, b, n, batch, stream);
}

int bigint_sub(uint32_t* out, uint32_t* borrow_out, const uint32_t* a, const uint32_t* b,
               int64_t n, int64_t batch, void* stream) {
  return addsub_common(true, out, borrow_out, a, b, n, batch, stream);
}

static bool mfma_fits(int64_t na, int64_t nb, MfmaCfg cfg) {
  return na <= BIGINT_MFMA_MAX_LIMBS && nb <= BIGINT_MFMA_MAX_LIMBS &&
         mfma_lds((int)na, (int)nb, cfg) <= 163840;
}

// a configuration forced on this thread keeps one work-group per instance
static bool split_forced() { return t_cfg_P || t_cfg_waves || t_cfg_dw || t_cfg_tile; }

// products of a small batch with each product's bands split over `parts`
// work-groups: carry words in a stream-ordered workspace, two launches
static int mul_split(uint32_t* out, const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, int nout,
                     int64_t batch, int dw, int parts, int wstride, hipStream_t s) {
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, (size_t)batch * wstride * 8, s);
  if (e != hipSuccess) { set_hip_error(e); return BIGINT_ENOMEM; }
  const int rc = launch_mul_mfma_split(out, a, na, b, nb, nout, batch, dw, parts,
                                       reinterpret_cast<uint64_t*>(ws), wstride, s);
  e = hipFreeAsync(ws, s);
  if (rc != BIGINT_OK) return rc;
  if (e != hipSuccess) { set_hip_error(e); return BIGINT_EHIP; }
  return BIGINT_OK;
}

int bigint_mul(uint32_t* out, const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb,
               int64_t batch, int algo, void* stream) {
  if (!out || !a || !b || na <= 0 || nb <= 0 || batch < 0) return BIGINT_EINVAL;
  if (algo != BIGINT_MUL_AUTO && algo != BIGINT_MUL_PLAIN && algo != BIGINT_MUL_MFMA &&
      algo != BIGINT_MUL_KARATSUBA)
    return BIGINT_EINVAL;
  if (batch > 0x7fffffff || na > (1 << 20) || nb > (1 << 20)) return BIGINT_EUNSUPPORTED;
  const size_t ob = (size_t)(na + nb) * batch * 4;
  if (overlap(out, ob, a, (size_t)na * batch * 4) || overlap(out, ob, b, (size_t)nb * batch * 4))
    return BIGINT_EINVAL;
  if (algo == BIGINT_MUL_KARATSUBA) {
    if (na != nb || na < 2) return BIGINT_EUNSUPPORTED;
    const int h = (int)((na + 1) / 2);
    MfmaCfg hc = current_mfma_cfg(h, h);
    if (hc.waves == 1) hc.waves = 4;   // the half products run one per work-group
    hc.tile = 16;                      // on 16x16 tiles
    if (!mfma_fits(h, h, hc)) return BIGINT_EUNSUPPORTED;
    if (batch == 0) return BIGINT_OK;
    BI_DEBUG("bigint: mul %lld x (%lld x %lld limbs): one Karatsuba level, half products of %d limbs "
             "with %d-bit digits, %d strips per band, %d waves\n",
             (long long)batch, (long long)na, (long long)nb, h, hc.dw, hc.P, hc.waves);
    hipStream_t s = (hipStream_t)stream;
    void* ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, kara_ws_bytes((int)na, batch), s);
    if (e != hipSuccess) { set_hip_error(e); return BIGINT_ENOMEM; }
    const int rc = launch_mul_kara(out, a, b, na, batch, ws, hc, s);
    e = hipFreeAsync(ws, s);
    if (rc != BIGINT_OK) return rc;
    if (e != hipSuccess) { set_hip_error(e); return BIGINT_EHIP; }
    return BIGINT_OK;
  }
  const MfmaCfg cfg = uniform_mfma_cfg((int)na, (int)nb, batch, false);
  int use = algo;
  if (use == BIGINT_MUL_AUTO)
    use = (mfma_fits(na, nb, cfg) && std::min(na, nb) >= 64) ? BIGINT_MUL_MFMA : BIGINT_MUL_PLAIN;
  if (use == BIGINT_MUL_MFMA) {
    if (!mfma_fits(na, nb, cfg)) return BIGINT_EUNSUPPORTED;
    if (batch == 0) return BIGINT_OK;
    // fewer instances than CUs and no configuration forced: each product's
    // bands split over several work-groups
    int wstride = 0;
    const int nout = (int)(na + nb);
    const int parts = split_forced() ? 1 : mul_mfma_split_parts((int)na, (int)nb, nout, batch, cfg.dw, &wstride);
    BI_DEBUG("bigint: mul %lld x (%lld x %lld limbs): MFMA-split, %d-bit digits, %dx%d tiles, %d strips "
             "per band, %d waves, %d work-group(s) per product\n",
             (long long)batch, (long long)na, (long long)nb, cfg.dw, cfg.tile, cfg.tile,
             parts > 1 ? 4 : cfg.P, parts > 1 ? 4 : cfg.waves, parts);
    if (parts > 1)
      return mul_split(out, a, na, b, nb, nout, batch, cfg.dw, parts, wstride, (hipStream_t)stream);
    return launch_mul_mfma(out, nullptr, a, na, b, nb, batch, cfg, (hipStream_t)stream);
  }
  if (na + nb > 32768) return BIGINT_EUNSUPPORTED;
  if (batch == 0) return BIGINT_OK;
  BI_DEBUG("bigint: mul %lld x (%lld x %lld limbs): plain u64 kernel\n", (long long)batch, (long long)na,
           (long long)nb);
  return launch_mul_plain(out, a, na, b, nb, batch, (hipStream_t)stream);
}

int bigint_mfma_split_parts(int64_t na, int64_t nb, int64_t batch, int* parts) {
  if (na <= 0 || nb <= 0 || batch < 1 || !parts) return BIGINT_EINVAL;
  *parts = 1;
  if (na > BIGINT_MFMA_MAX_LIMBS || nb > BIGINT_MFMA_MAX_LIMBS) return BIGINT_OK;
  const MfmaCfg cfg = uniform_mfma_cfg((int)na, (int)nb, batch, false);
  if (!mfma_fits(na, nb, cfg) || split_forced()) return BIGINT_OK;
  int wstride = 0;
  *parts = mul_mfma_split_parts((int)na, (int)nb, (int)(na + nb), batch, cfg.dw, &wstride);
  return BIGINT_OK;
}

int bigint_mullo(uint32_t* out, const uint32_t* a, const uint32_t* b, int64_t n, int64_t batch,
                 void* stream) {
  if (!out || !a || !b || n <= 0 || batch < 0) return BIGINT_EINVAL;
  if (batch > 0x7fffffff || n > BIGINT_MFMA_MAX_LIMBS) return BIGINT_EUNSUPPORTED;
  const size_t bytes = (size_t)n * batch * 4;
  if (overlap(out, bytes, a, bytes) || overlap(out, bytes, b, bytes)) return BIGINT_EINVAL;
  const MfmaCfg cfg = uniform_mfma_cfg((int)n, (int)n, batch, true);
  if (!mfma_fits(n, n, cfg)) return BIGINT_EUNSUPPORTED;
  if (batch == 0) return BIGINT_OK;
  int wstride = 0;
  const int parts = split_forced() ? 1 : mul_mfma_split_parts((int)n, (int)n, (int)n, batch, cfg.dw, &wstride);
  if (parts > 1) return mul_split(out, a, n, b, n, (int)n, batch, cfg.dw, parts, wstride, (hipStream_t)stream);
  return launch_mul_mfma(out, nullptr, a, n, b, n, batch, cfg, (hipStream_t)stream, (int)n);
}

int bigint_add6(uint32_t* out, uint32_t* overflow, const uint32_t* a, const uint32_t* b,
                int64_t n, int64_t batch, void* stream) {
  if (!out || !a || !b || n <= 0 || batch < 0) return BIGINT_EINVAL;
  if (n > 16384 || batch > 0x7fffffff) return BIGINT_EUNSUPPORTED;
  const size_t bytes = (size_t)n * batch * 4;
  if (out != a && overlap(out, bytes, a, bytes)) return BIGINT_EINVAL;
  if (out != b && overlap(out, bytes, b, bytes)) return BIGINT_EINVAL;
  if (overflow) {
    const size_t cb = (size_t)batch * 4;
    if (overlap(overflow, cb, out, bytes) || overlap(overflow, cb, a, bytes) ||
        overlap(overflow, cb, b, bytes))
      return BIGINT_EINVAL;
  }
  if (batch == 0) return BIGINT_OK;
  return launch_add6(out, overflow, a, b, n, batch, (hipStream_t)stream);
}

int bigint_poly(uint32_t* out, const uint32_t* a, const uint32_t* b, int64_t n, int64_t batch,
                void* stream) {
  if (!out || !a || !b || n <= 0 || batch < 0) return BIGINT_EINVAL;
  if (batch > 0x7fffffff || n > BIGINT_MFMA_MAX_LIMBS) return BIGINT_EUNSUPPORTED;
  const size_t bytes = (size_t)n * batch * 4;
  if (overlap(out, bytes, a, bytes) || overlap(out, bytes, b, bytes)) return BIGINT_EINVAL;
  MfmaCfg cfg = default_mfma_cfg((int)n, (int)n);
  cfg.dw = 8;
  cfg.tile = 16;   // Poly's kernels run 16x16 tiles
  if (cfg.waves == 1 && mfma_wave_fits(n, n) && wave_batch(n, n, batch, kWavePoly)) {
    // small operands in large batches: one wave per instance, like the products
    if (batch == 0) return BIGINT_OK;
    const int P = cfg.P == 4 ? 4 : 8;
    const int chunk = poly_wave_chunk((int)n, batch, P);
    hipStream_t s = (hipStream_t)stream;
    void* ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, (size_t)chunk * 2 * n * 4, s);
    if (e != hipSuccess) { set_hip_error(e); return BIGINT_ENOMEM; }
    const int rc = launch_poly_wave(out, a, b, n, batch, (uint32_t*)ws, chunk, P, s);
    e = hipFreeAsync(ws, s);
    if (rc != BIGINT_OK) return rc;
    if (e != hipSuccess) { set_hip_error(e); return BIGINT_EHIP; }
    return BIGINT_OK;
  }
  if (cfg.waves == 1) cfg = MfmaCfg{4, 4, 8};   // the work-group kernel, as for products mod B^n
  if (poly_lds((int)n, cfg) > 163840) return BIGINT_EUNSUPPORTED;
  if (batch == 0) return BIGINT_OK;
  // launches of `grid` work-groups, each owning 2n limbs of workspace
  const int grid = poly_chunk((int)n, batch, cfg);
  hipStream_t s = (hipStream_t)stream;
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, (size_t)grid * 2 * n * 4, s);
  if (e != hipSuccess) { set_hip_error(e); return BIGINT_ENOMEM; }
  const int rc = launch_poly(out, a, b, n, batch, (uint32_t*)ws, grid, cfg, s);
  e = hipFreeAsync(ws, s);
  if (rc != BIGINT_OK) return rc;
  if (e != hipSuccess) { set_hip_error(e); return BIGINT_EHIP; }
  return BIGINT_OK;
}

int bigint_digits7(uint8_t* out, const uint32_t* a, int64_t n, int64_t D, int64_t batch,
                   void* stream) {
  if (!out || !a || n <= 0 || D <= 0 || batch < 0) return BIGINT_EINVAL;
  if (batch > 0xffff || n > (1 << 24) || D > (1 << 26)) return BIGINT_EUNSUPPORTED;
  if (overlap(out, (size_t)D * batch, a, (size_t)n * batch * 4)) return BIGINT_EINVAL;
  if (batch == 0) return BIGINT_OK;
  return launch_digits7(out, a, n, D, batch, (hipStream_t)stream);
}

int bigint_conv7(int32_t* c, const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb,
                 int64_t batch, void* stream) {
  if (!c || !a || !b || na <= 0 || nb <= 0 || batch < 0) return BIGINT_EINVAL;
  MfmaCfg cfg = current_mfma_cfg((int)na, (int)nb);
  cfg.dw = 7;  // the raw coefficients are those of the 7-bit digits
  cfg.tile = 16;
  if (!mfma_fits(na, nb, cfg) || batch > 0x7fffffff) return BIGINT_EUNSUPPORTED;
  const int64_t K = (32 * na + 6) / 7 + (32 * nb + 6) / 7 - 1;
  const size_t cb = (size_t)K * batch * 4;
  if (overlap(c, cb, a, (size_t)na * batch * 4) || overlap(c, cb, b, (size_t)nb * batch * 4))
    return BIGINT_EINVAL;
  if (batch == 0) return BIGINT_OK;
  return launch_mul_mfma(nullptr, c, a, na, b, nb, batch, cfg, (hipStream_t)stream);
}

}  // extern "C"

// ============================================================================
// plans and ragged batches
// ============================================================================
struct bigint_plan_s {
  int op = 0, flags = 0;
  int64_t batch = 0;
  std::vector<int64_t> la, lb;
  // schedule: the queue (largest first; division: int32 instance indices)
  bi::QueueItem* d_queue = nullptr;
  std::vector<bi::RaggedClass> cls;  // MFMA multiply: one launch per segment
  // per segment (bigint_plan_segments): digit products its instances compute,
  // and its modelled busy fraction (sum of costs / (slots x list-schedule span))
  std::vector<int64_t> seg_products;
  std::vector<double> seg_busy;
  std::vector<int> seg_slots;
  size_t lds = 0;                    // plain multiply
  bool plain = false;
  int grid = 0;               // division: work-groups (workspace slots) per launch
  int cap_u = 0, cap_v = 0;   // division: largest dividend / divisor
  // workspace
  void* ws = nullptr;
  size_t ws_bytes = 0, ws_need = 0;
  bool ws_owned = false;
  // graph replay keyed by the call's pointers
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* key[9] = {};
  // counters reported by bigint_plan_info
  int64_t n_launches = 0;     // kernel launches one call enqueues
  int64_t n_captures = 0;     // graphs instantiated so far
  int64_t n_replays = 0;      // calls served by launching an instantiated graph
};

// Runs launch(stream) through the plan's hipGraph: captured on the plan's own
// stream the first time (and whenever the call's pointers change), then
// launched on the caller's stream, the null stream included.
template <class F>
static int plan_graph_call(bigint_plan_s* plan, const void* const* key, int nkey, F launch,
                           hipStream_t s) {
  if (memcmp(key, plan->key, sizeof(void*) * nkey) != 0 || !plan->exec) {
    if (plan->exec) { (void)hipGraphExecDestroy(plan->exec); plan->exec = nullptr; }
    if (plan->graph) { (void)hipGraphDestroy(plan->graph); plan->graph = nullptr; }
    if (!plan->cap_stream) BI_HIP(hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking));
    BI_HIP(hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = launch(plan->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(plan->cap_stream, &g);
    if (rc != BIGINT_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) { set_hip_error(e); return BIGINT_EHIP; }
    plan->graph = g;
    BI_HIP(hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0));
    memset(plan->key, 0, sizeof(plan->key));
    memcpy(plan->key, key, sizeof(void*) * nkey);
    ++plan->n_captures;
  } else {
    ++plan->n_replays;
  }
  BI_HIP(hipGraphLaunch(plan->exec, s));
  return BIGINT_OK;
}

static int plan_build_mul(bigint_plan_s* p) {
  const int64_t B = p->batch;
  bool plain = (p->flags & BIGINT_PLAN_PLAIN) != 0;
  for (int64_t i = 0; i < B && !plain; ++i) {
    const MfmaCfg c = ragged_mfma_cfg((int)p->la[i], (int)p->lb[i]);
    if (!mfma_fits(p->la[i], p->lb[i], c) || std::min(p->la[i], p->lb[i]) < 1) plain = true;
  }
  for (int64_t i = 0; i < B; ++i)
    if (plain && p->la[i] + p->lb[i] > 32768) return BIGINT_EUNSUPPORTED;
  p->plain = plain;
  // largest first (cost ~ digit products), ties by index
  auto cost = [&](int64_t i) { return p->la[i] * p->lb[i]; };
  std::vector<int64_t> idx(B);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return cost(x) > cost(y); });
  std::vector<QueueItem> q(B);
  if (plain) {
    size_t lds = 0;
    for (int64_t t = 0; t < B; ++t) {
      q[t] = QueueItem{(int32_t)idx[t], 0};
      lds = std::max(lds, plain_lds((int)p->la[idx[t]], (int)p->lb[idx[t]]));
    }
    p->lds = lds;
  } else {
    // Segments, one launch each.  A segment starts with the largest remaining
    // instance; its core is the run of instances with the same digit width,
    // waves and LDS-bound work-groups per CU and no more strips per band (the
    // segment's kernel runs those with fewer strips inlined; one launch over
    // them balances better than a launch per strips-per-band value: 4096
    // ragged products 2.18 -> 2.12 ms).  The core is
    // list-scheduled largest first on the launch's resident work-groups (as
    // in-order dispatch will run it); then the following instances of the
    // same digit width and no more strips per band join the segment as long
    // as each fits in the idle time before the core's last work-group ends.
    struct It {
      int64_t i;
      MfmaCfg c;
      int lpc;  // work-groups per CU its LDS and the kernel's registers allow
    };
    // work-groups per CU the registers allow, per (configuration, waves)
    std::vector<std::pair<int, int>> occ_key;
    std::vector<int> occ_val;
    auto reg_occ = [&](int id, int waves) {
      for (size_t j = 0; j < occ_key.size(); ++j)
        if (occ_key[j] == std::make_pair(id, waves)) return occ_val[j];
      const int v = std::max(1, ragged_slots(id, waves, 1024) / std::max(1, num_cus()));
      occ_key.emplace_back(id, waves);
      occ_val.push_back(v);
      return v;
    };
    std::vector<It> it(B);
    for (int64_t t = 0; t < B; ++t) {
      const int64_t i = idx[t];
      const MfmaCfg c = ragged_mfma_cfg((int)p->la[i], (int)p->lb[i]);
      const size_t l = mfma_lds((int)p->la[i], (int)p->lb[i], c);
      const int by_lds = (int)std::min<size_t>(4, 163840 / std::max<size_t>(l, 1));
      it[t] = It{i, c, std::min(by_lds, reg_occ(ragged_cfg_id(c), c.waves))};
    }
    std::vector<RaggedClass> cls;
    int64_t pos = 0;
    while (pos < B) {
      const It& h = it[pos];
      RaggedClass k{ragged_cfg_id(h.c), h.c.waves, (int)pos, 0, 0};
      int64_t end = pos;
      while (end < B && it[end].c.P <= h.c.P && it[end].c.dw == h.c.dw &&
             it[end].c.waves == h.c.waves && it[end].lpc == h.lpc) {
        const int64_t i = it[end].i;
        // (each instance's own strips per band: fewer strips, more bands)
        k.lds = std::max(k.lds, mfma_lds((int)p->la[i], (int)p->lb[i],
                                         MfmaCfg{it[end].c.P, k.waves, h.c.dw}));
        ++end;
      }
      const int slots = ragged_slots(k.cfg, k.waves, k.lds);
      if (slots < 1) return BIGINT_EUNSUPPORTED;
      std::priority_queue<double, std::vector<double>, std::greater<double>> fin;
      for (int m = 0; m < slots; ++m) fin.push(0.0);
      double span = 0.0;
      for (int64_t t = pos; t < end; ++t) {
        const double f = fin.top() + (double)cost(it[t].i);
        fin.pop();
        fin.push(f);
        span = std::max(span, f);
      }
      while (end < B) {
        const It& f = it[end];
        if (f.c.dw != h.c.dw || f.c.P > h.c.P) break;
        const MfmaCfg fc{f.c.P, k.waves, f.c.dw};
        if (mfma_lds((int)p->la[f.i], (int)p->lb[f.i], fc) > k.lds) break;
        const double t0 = fin.top() + (double)cost(f.i);
        if (t0 > span) break;
        fin.pop();
        fin.push(t0);
        ++end;
      }
      k.count = (int)(end - pos);
      double work = 0.0, fspan = 0.0;
      int64_t prod = 0;
      for (int64_t t = pos; t < end; ++t) {
        q[t] = QueueItem{(int32_t)it[t].i, it[t].c.P};
        work += (double)cost(it[t].i);
        const int64_t i = it[t].i;
        const int64_t da = h.c.dw == 8 ? 4 * p->la[i] : (32 * p->la[i] + 6) / 7;
        const int64_t db = h.c.dw == 8 ? 4 * p->lb[i] : (32 * p->lb[i] + 6) / 7;
        prod += da * db;
      }
      while (!fin.empty()) { fspan = std::max(fspan, fin.top()); fin.pop(); }
      p->seg_products.push_back(prod);
      p->seg_busy.push_back(fspan > 0.0 ? work / ((double)slots * fspan) : 0.0);
      p->seg_slots.push_back(slots);
      BI_DEBUG("bigint: plan segment %zu: %d products from queue position %d, %d-bit digits, %d strips "
               "per band, %d waves, %zu bytes of LDS, %d resident work-groups, modelled busy %.3f\n",
               cls.size(), k.count, k.first, h.c.dw, h.c.P, k.waves, k.lds, slots, p->seg_busy.back());
      cls.push_back(k);
      pos = end;
    }
    // A segment of few instances leaves most CUs idle however it is
    // ordered: split every instance's bands over several work-groups, as a
    // small uniform batch is (parts: enough to fill the CUs once, at most a
    // quarter of the largest instance's 4-strip bands, at least four), with
    // the strips' carry words in the plan's workspace.
    const int R = num_cus();
    int64_t ws_words = 0;
    for (RaggedClass& k : cls) {
      if ((int64_t)k.count * 4 > R) continue;
      const int dw = k.cfg >= 3 ? 8 : 7;
      int wmax = 0, w0 = 0;
      size_t lmax = 0;
      for (int t = k.first; t < k.first + k.count; ++t) {
        const int64_t i = q[t].inst;
        int w;
        size_t l;
        ragged_split_geo((int)p->la[i], (int)p->lb[i], dw, &w, &l);
        if (t == k.first) w0 = w;   // the largest instance
        wmax = std::max(wmax, w);
        lmax = std::max(lmax, l);
      }
      const int nb0 = (w0 + 3) / 4;   // 4-strip bands of the largest instance
      const int parts = (int)std::min<int64_t>((R + k.count - 1) / k.count, nb0 / 4);
      if (nb0 < 32 || parts < 4 || lmax > 163840) continue;
      k.parts = parts;
      BI_DEBUG("bigint: plan segment of %d products from queue position %d split: %d work-groups per "
               "product\n", k.count, k.first, parts);
      k.wstride = wmax;
      k.split_lds = lmax;
      k.ws_off = ws_words;
      ws_words += (int64_t)k.count * wmax;
    }
    p->cls = cls;
    p->ws_need = (size_t)ws_words * 8;
  }
  p->n_launches = 0;
  if (plain) p->n_launches = B > 0 ? 1 : 0;
  for (const RaggedClass& k : p->cls) p->n_launches += k.parts > 1 ? 2 : 1;
  if (B > 0) {
    BI_HIP(hipMalloc(&p->d_queue, sizeof(QueueItem) * B));
    BI_HIP(hipMemcpy(p->d_queue, q.data(), sizeof(QueueItem) * B, hipMemcpyHostToDevice));
  }
  if (plain || B == 0) p->ws_need = 0;  // otherwise set with the segments
  return BIGINT_OK;
}

static int plan_build_div(bigint_plan_s* p) {
  const int64_t B = p->batch;
  int64_t cu = 1, cv = 1;
  for (int64_t i = 0; i < B; ++i) {
    if (p->la[i] > BIGINT_DIV_MAX_LIMBS || p->lb[i] > BIGINT_DIV_MAX_LIMBS) return BIGINT_EUNSUPPORTED;
    cu = std::max(cu, p->la[i]);
    cv = std::max(cv, p->lb[i]);
  }
  p->cap_u = (int)cu;
  p->cap_v = (int)cv;
  // largest first: the cost grows like (nu - nv) (nu + 4 nv) limb products
  std::vector<int64_t> idx(B);
  std::iota(idx.begin(), idx.end(), 0);
  auto cost = [&](int64_t i) {
    const int64_t d = std::max<int64_t>(p->la[i] - p->lb[i] + 1, 1);
    return d * (p->la[i] + 4 * p->lb[i]);
  };
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return cost(x) > cost(y); });
  std::vector<int32_t> q(B);
  for (int64_t t = 0; t < B; ++t) q[t] = (int32_t)idx[t];
  // The work-groups resident at the start land one per CU in rows: work-
  // group j and j + R (R CUs) share a CU.  Reversing every other row (a
  // snake over the largest-first order) pairs each of the largest divisions
  // with one of the smallest, so the divisions that set the call's time
  // share their CU the least (512 divisions of 2^16..2^18 bits: 0.402 ->
  // 0.380 ms; pairing neighbours in the order instead: 0.45 ms).
  {
    const int64_t R = num_cus();
    const int64_t e = std::min<int64_t>(B, R * div_groups_per_cu(p->cap_u, p->cap_v));
    for (int64_t row = 1; row * R < e; row += 2)
      std::reverse(q.begin() + row * R, q.begin() + std::min(e, (row + 1) * R));
  }
  p->grid = div_chunk(p->cap_u, p->cap_v, B);
  p->n_launches = B > 0 ? (B + p->grid - 1) / p->grid : 0;
  BI_DEBUG("bigint: plan of %lld divisions: dividends up to %d limbs, divisors up to %d, %d threads per "
           "division, %d per CU, %d per launch\n",
           (long long)B, p->cap_u, p->cap_v, div_threads(p->cap_u), div_groups_per_cu(p->cap_u, p->cap_v),
           p->grid);
  if (B > 0) {
    BI_HIP(hipMalloc(&p->d_queue, sizeof(int32_t) * B));
    BI_HIP(hipMemcpy(p->d_queue, q.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice));
  }
  p->ws_need = div_ws_bytes(p->cap_u, p->cap_v, p->grid);
  if (div_lds_bytes(p->cap_u, p->cap_v) > 163840 - 256) return BIGINT_EUNSUPPORTED;
  return BIGINT_OK;
}

static void plan_free(bigint_plan_s* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->d_queue) (void)hipFree(p->d_queue);
  if (p->ws_owned && p->ws) (void)hipFree(p->ws);
  delete p;
}

extern "C" {

int bigint_plan_create(bigint_plan_t* plan, int op, const int64_t* len_a, const int64_t* len_b,
                       int64_t batch, int flags) {
  if (!plan) return BIGINT_EINVAL;
  *plan = nullptr;
  if (batch < 0 || (batch > 0 && (!len_a || !len_b))) return BIGINT_EINVAL;
  if (op != BIGINT_OP_MUL && op != BIGINT_OP_DIVMOD) return BIGINT_EINVAL;
  if (flags & ~(BIGINT_PLAN_PLAIN | BIGINT_PLAN_NO_GRAPH)) return BIGINT_EINVAL;
  if (batch > 0x7fffffff) return BIGINT_EUNSUPPORTED;
  for (int64_t i = 0; i < batch; ++i)
    if (len_a[i] <= 0 || len_b[i] <= 0) return BIGINT_EINVAL;
  bigint_plan_s* p = new (std::nothrow) bigint_plan_s;
  if (!p) return BIGINT_ENOMEM;
  p->op = op;
  p->flags = flags;
  p->batch = batch;
  p->la.assign(len_a, len_a + batch);
  p->lb.assign(len_b, len_b + batch);
  int rc = BIGINT_OK;
  if (op == BIGINT_OP_MUL) rc = plan_build_mul(p);
  else rc = plan_build_div(p);
  if (rc != BIGINT_OK) { plan_free(p); return rc; }
  *plan = p;
  return BIGINT_OK;
}

int bigint_plan_workspace_size(bigint_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return BIGINT_EINVAL;
  *bytes = plan->ws_need;
  return BIGINT_OK;
}

int bigint_plan_set_workspace(bigint_plan_t plan, void* dev, size_t bytes) {
  if (!plan || (!dev && bytes)) return BIGINT_EINVAL;
  if (bytes < plan->ws_need) return BIGINT_EINVAL;
  if (plan->ws_owned && plan->ws) (void)hipFree(plan->ws);
  plan->ws = dev;
  plan->ws_bytes = bytes;
  plan->ws_owned = false;
  return BIGINT_OK;
}

int bigint_plan_destroy(bigint_plan_t plan) {
  if (!plan) return BIGINT_EINVAL;
  plan_free(plan);
  return BIGINT_OK;
}

int bigint_plan_info(bigint_plan_t plan, int64_t* info, int n) {
  if (!plan || (!info && n > 0) || n < 0) return BIGINT_EINVAL;
  const int64_t v[3] = {plan->n_launches, plan->n_captures, plan->n_replays};
  for (int i = 0; i < n; ++i) info[i] = i < 3 ? v[i] : 0;
  return BIGINT_OK;
}

int bigint_plan_segments(bigint_plan_t plan, int64_t* seg, int max_segments, int* n_segments) {
  if (!plan || !n_segments || max_segments < 0 || (!seg && max_segments > 0)) return BIGINT_EINVAL;
  const bool mfma = plan->op == BIGINT_OP_MUL && !plan->plain;
  const int n = mfma ? (int)plan->cls.size() : 0;
  *n_segments = n;
  for (int k = 0; k < std::min(n, max_segments); ++k) {
    const RaggedClass& c = plan->cls[k];
    int64_t* o = seg + 9 * k;
    o[0] = c.first;
    o[1] = c.count;
    o[2] = c.cfg >= 3 ? 8 : 7;
    o[3] = 4 << (c.cfg % 3);
    o[4] = c.waves;
    o[5] = plan->seg_slots[k];
    o[6] = plan->seg_products[k];
    o[7] = (int64_t)std::llround(1e6 * plan->seg_busy[k]);
    o[8] = c.parts;
  }
  return BIGINT_OK;
}

static int ragged_mul_checks(uint32_t* out, const int64_t* out_off, const uint32_t* a,
                             const int64_t* a_off, const uint32_t* b, const int64_t* b_off,
                             int64_t batch, bigint_plan_t plan) {
  if (!plan || plan->op != BIGINT_OP_MUL || batch != plan->batch) return BIGINT_EINVAL;
  if (batch == 0) return BIGINT_OK;
  if (!out || !out_off || !a || !a_off || !b || !b_off) return BIGINT_EINVAL;
  int64_t ta = 0, tb = 0;
  for (int64_t i = 0; i < batch; ++i) { ta += plan->la[i]; tb += plan->lb[i]; }
  const size_t ob = (size_t)(ta + tb) * 4;
  if (overlap(out, ob, a, (size_t)ta * 4) || overlap(out, ob, b, (size_t)tb * 4)) return BIGINT_EINVAL;
  return BIGINT_OK;
}

// the plan's workspace, allocated (and owned) on first use if none was set
static int plan_ws(bigint_plan_t plan) {
  if (plan->ws_need == 0 || plan->ws) return BIGINT_OK;
  BI_HIP(hipMalloc(&plan->ws, plan->ws_need));
  plan->ws_bytes = plan->ws_need;
  plan->ws_owned = true;
  return BIGINT_OK;
}

int bigint_mul_ragged_segment(uint32_t* out, const int64_t* out_off, const uint32_t* a,
                              const int64_t* a_off, const uint32_t* b, const int64_t* b_off,
                              int64_t batch, bigint_plan_t plan, int segment, void* stream) {
  int rc = ragged_mul_checks(out, out_off, a, a_off, b, b_off, batch, plan);
  if (rc != BIGINT_OK) return rc;
  if (plan->plain || segment < 0 || segment >= (int)plan->cls.size()) return BIGINT_EINVAL;
  if ((rc = plan_ws(plan)) != BIGINT_OK) return rc;
  return launch_mul_ragged(out, out_off, a, a_off, b, b_off, plan->d_queue, plan->cls.data() + segment,
                           1, plan->ws, (hipStream_t)stream);
}

int bigint_mul_ragged(uint32_t* out, const int64_t* out_off, const uint32_t* a,
                      const int64_t* a_off, const uint32_t* b, const int64_t* b_off, int64_t batch,
                      bigint_plan_t plan, void* stream) {
  int rc = ragged_mul_checks(out, out_off, a, a_off, b, b_off, batch, plan);
  if (rc != BIGINT_OK || batch == 0) return rc;
  if ((rc = plan_ws(plan)) != BIGINT_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  auto launch = [&](hipStream_t ls) {
    if (plan->plain)
      return launch_mul_plain_ragged(out, out_off, a, a_off, b, b_off, plan->d_queue, batch,
                                     plan->lds, ls);
    return launch_mul_ragged(out, out_off, a, a_off, b, b_off, plan->d_queue, plan->cls.data(),
                             (int)plan->cls.size(), plan->ws, ls);
  };
  if (plan->flags & BIGINT_PLAN_NO_GRAPH) return launch(s);
  const void* key[7] = {out, out_off, a, a_off, b, b_off, plan->ws};
  return plan_graph_call(plan, key, 7, launch, s);
}

// ---- division ------------------------------------------------------------------

static int divmod_launch_alloc(uint32_t* q, uint32_t* r, int32_t* status, const uint32_t* u,
                               int64_t nu, const uint32_t* v, int64_t nv, int64_t batch, int h_inv,
                               hipStream_t s) {
  const int cap_u = h_inv >= 0 ? h_inv + 2 : (int)nu;
  const int cap_v = (int)nv;
  const int grid = div_chunk(cap_u, cap_v, batch);
  const size_t bytes = div_ws_bytes(cap_u, cap_v, grid);
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, bytes, s);
  if (e != hipSuccess) { set_hip_error(e); return BIGINT_ENOMEM; }
  const int rc = launch_divmod(q, nullptr, r, nullptr, status, u, nullptr, (int)nu, v, nullptr,
                               (int)nv, nullptr, batch, ws, cap_u, cap_v, grid, h_inv, nullptr, s);
  e = hipFreeAsync(ws, s);
  if (rc != BIGINT_OK) return rc;
  if (e != hipSuccess) { set_hip_error(e); return BIGINT_EHIP; }
  return BIGINT_OK;
}

int bigint_divmod(uint32_t* q, uint32_t* r, int32_t* status, const uint32_t* u, int64_t nu,
                  const uint32_t* v, int64_t nv, int64_t batch, void* stream) {
  if (!q || !r || !u || !v || nu <= 0 || nv <= 0 || batch < 0) return BIGINT_EINVAL;
  if (nu > BIGINT_DIV_MAX_LIMBS || nv > BIGINT_DIV_MAX_LIMBS || batch > 0x7fffffff)
    return BIGINT_EUNSUPPORTED;
  const size_t qb = (size_t)nu * batch * 4, rb = (size_t)nv * batch * 4;
  const size_t ub = (size_t)nu * batch * 4, vb = (size_t)nv * batch * 4, sb = (size_t)batch * 4;
  if (overlap(q, qb, u, ub) || overlap(q, qb, v, vb) || overlap(r, rb, u, ub) ||
      overlap(r, rb, v, vb) || overlap(q, qb, r, rb))
    return BIGINT_EINVAL;
  if (status && (overlap(status, sb, q, qb) || overlap(status, sb, r, rb) ||
                 overlap(status, sb, u, ub) || overlap(status, sb, v, vb)))
    return BIGINT_EINVAL;
  if (batch == 0) return BIGINT_OK;
  return divmod_launch_alloc(q, r, status, u, nu, v, nv, batch, -1, (hipStream_t)stream);
}

int bigint_divmod_noalloc(uint32_t* q, uint32_t* r, int32_t* status, const uint32_t* u, int64_t nu,
                          const uint32_t* v, int64_t nv, int64_t batch, void* stream) {
  if (!q || !r || !u || !v || nu <= 0 || nv <= 0 || batch < 0) return BIGINT_EINVAL;
  if (nu > BIGINT_DIV_MAX_LIMBS || nv > BIGINT_DIV_MAX_LIMBS || batch > 0x7fffffff)
    return BIGINT_EUNSUPPORTED;
  const size_t qb = (size_t)nu * batch * 4, rb = (size_t)nv * batch * 4;
  const size_t ub = (size_t)nu * batch * 4, vb = (size_t)nv * batch * 4, sb = (size_t)batch * 4;
  if (overlap(q, qb, u, ub) || overlap(q, qb, v, vb) || overlap(r, rb, u, ub) ||
      overlap(r, rb, v, vb) || overlap(q, qb, r, rb))
    return BIGINT_EINVAL;
  if (status && (overlap(status, sb, q, qb) || overlap(status, sb, r, rb) ||
                 overlap(status, sb, u, ub) || overlap(status, sb, v, vb)))
    return BIGINT_EINVAL;
  if (batch == 0) return BIGINT_OK;
  void* ws = nullptr;
  size_t cap = 0;
  const int rc = div_scratch(&ws, &cap);
  if (rc != BIGINT_OK) return rc;
  // work-groups per launch: as bigint_divmod, but no more workspace slots
  // than the scratch array holds (the launches run one after another)
  const size_t slot = div_ws_bytes((int)nu, (int)nv, 1);
  const int64_t grid = std::min<int64_t>(div_chunk((int)nu, (int)nv, batch), (int64_t)(cap / slot));
  if (grid < 1) return BIGINT_EUNSUPPORTED;
  return launch_divmod(q, nullptr, r, nullptr, status, u, nullptr, (int)nu, v, nullptr, (int)nv,
                       nullptr, batch, ws, (int)nu, (int)nv, (int)grid, -1, nullptr,
                       (hipStream_t)stream);
}

int bigint_shinv(uint32_t* w, const uint32_t* v, int64_t nv, int64_t h, int64_t batch,
                 void* stream) {
  if (!w || !v || nv <= 0 || batch < 0 || h < nv) return BIGINT_EINVAL;
  if (h > BIGINT_DIV_MAX_LIMBS || batch > 0x7fffffff) return BIGINT_EUNSUPPORTED;
  if (overlap(w, (size_t)(h + 1) * batch * 4, v, (size_t)nv * batch * 4)) return BIGINT_EINVAL;
  if (batch == 0) return BIGINT_OK;
  return divmod_launch_alloc(w, nullptr, nullptr, nullptr, nv, v, nv, batch, (int)h,
                             (hipStream_t)stream);
}

static int divmod_ragged(uint32_t* q, const int64_t* q_off, uint32_t* r, const int64_t* r_off,
                         int32_t* status, const uint32_t* u, const int64_t* u_off,
                         const uint32_t* v, const int64_t* v_off, int64_t batch,
                         bigint_plan_t plan, int64_t* counts, hipStream_t s) {
  if (!plan || plan->op != BIGINT_OP_DIVMOD || batch != plan->batch) return BIGINT_EINVAL;
  if (batch == 0) return BIGINT_OK;
  if (!q || !q_off || !r || !r_off || !u || !u_off || !v || !v_off) return BIGINT_EINVAL;
  int64_t tu = 0, tv = 0;
  for (int64_t i = 0; i < batch; ++i) { tu += plan->la[i]; tv += plan->lb[i]; }
  if (overlap(q, tu * 4, u, tu * 4) || overlap(q, tu * 4, v, tv * 4) || overlap(r, tv * 4, u, tu * 4) ||
      overlap(r, tv * 4, v, tv * 4) || overlap(q, tu * 4, r, tv * 4))
    return BIGINT_EINVAL;
  if (counts && (overlap(counts, (size_t)batch * 32, q, tu * 4) ||
                 overlap(counts, (size_t)batch * 32, r, tv * 4)))
    return BIGINT_EINVAL;
  if (!plan->ws) {
    BI_HIP(hipMalloc(&plan->ws, plan->ws_need));
    plan->ws_bytes = plan->ws_need;
    plan->ws_owned = true;
  }
  auto launch = [&](hipStream_t ls) {
    return launch_divmod(q, q_off, r, r_off, status, u, u_off, 0, v, v_off, 0,
                         reinterpret_cast<const int32_t*>(plan->d_queue), batch, plan->ws,
                         plan->cap_u, plan->cap_v, plan->grid, -1, counts, ls);
  };
  // the counting variant is a diagnostic: launched directly
  if (counts || (plan->flags & BIGINT_PLAN_NO_GRAPH)) return launch(s);
  const void* key[9] = {q, q_off, r, r_off, status, u, u_off, v, v_off};
  return plan_graph_call(plan, key, 9, launch, s);
}

int bigint_divmod_ragged(uint32_t* q, const int64_t* q_off, uint32_t* r, const int64_t* r_off,
                         int32_t* status, const uint32_t* u, const int64_t* u_off,
                         const uint32_t* v, const int64_t* v_off, int64_t batch,
                         bigint_plan_t plan, void* stream) {
  return divmod_ragged(q, q_off, r, r_off, status, u, u_off, v, v_off, batch, plan, nullptr,
                       (hipStream_t)stream);
}

int bigint_diag_divmod_ragged(int64_t* counts, uint32_t* q, const int64_t* q_off, uint32_t* r,
                              const int64_t* r_off, int32_t* status, const uint32_t* u,
                              const int64_t* u_off, const uint32_t* v, const int64_t* v_off,
                              int64_t batch, bigint_plan_t plan, void* stream) {
  if (!counts) return BIGINT_EINVAL;
  return divmod_ragged(q, q_off, r, r_off, status, u, u_off, v, v_off, batch, plan, counts,
                       (hipStream_t)stream);
}

int bigint_diag_mfma_rate(int32_t* scratch, int64_t blocks, int64_t iters, int toggle,
                          void* stream) {
  if (!scratch || blocks <= 0 || iters <= 0) return BIGINT_EINVAL;
  if (blocks > (1 << 20) || iters > (1 << 24)) return BIGINT_EUNSUPPORTED;
  return launch_mfma_rate(scratch, (int)blocks, (int)iters, toggle, (hipStream_t)stream);
}

int bigint_diag_mad_rate(uint64_t* scratch, int64_t blocks, int64_t iters, void* stream) {
  if (!scratch || blocks <= 0 || iters <= 0) return BIGINT_EINVAL;
  if (blocks > (1 << 20) || iters > (1 << 24)) return BIGINT_EUNSUPPORTED;
  return launch_mad_rate(scratch, (int)blocks, (int)iters, (hipStream_t)stream);
}

// ---- autotuning ------------------------------------------------------------------
// For each size bin, every tile configuration (strips per band P, waves per
// work-group, digit width) multiplies the same random batch; the fastest is
// kept.  All candidates must give identical bytes: every candidate's whole
// output is compared with the first one's on the device, and any difference
// fails the call (BIGINT_EHIP) without changing the table.

int bigint_autotune(const char* cache_path, int flags) {
  (void)flags;
  tune_env_once();
  static const int kBins[] = {128, 256, 512, 1024, 2048, 4096, 8192, 16384};
  static const int kP[] = {4, 8, 16, 32};
  static const int kW[] = {1, 4, 8};
  static const int kD[] = {7, 8};
  static const int kT[] = {16, 32};
  std::vector<TuneEntry> table;
  hipStream_t s = nullptr;
  BI_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BI_HIP(hipEventCreate(&e0));
  BI_HIP(hipEventCreate(&e1));
  int rc = BIGINT_OK;
  for (size_t bi_ = 0; bi_ < sizeof(kBins) / sizeof(kBins[0]) && rc == BIGINT_OK; ++bi_) {
    const int n = kBins[bi_];
    // enough instances to fill every CU several times: at least four per CU
    // (with fewer, configurations that fit two work-groups per CU leave
    // slots empty and lose to one-per-CU ones they beat on full batches)
    const double r = 16384.0 / n;
    const int nb = num_cus() * std::max(4, (int)(r * r / 8));
    const size_t in_bytes = (size_t)nb * n * 4, out_bytes = (size_t)nb * 2 * n * 4;
    uint32_t *a = nullptr, *b = nullptr, *out = nullptr;
    if (hipMalloc(&a, in_bytes) != hipSuccess || hipMalloc(&b, in_bytes) != hipSuccess ||
        hipMalloc(&out, out_bytes) != hipSuccess) {
      rc = BIGINT_ENOMEM;
    }
    // ref: the first candidate's whole output; every later candidate must
    // reproduce it byte for byte (compared on the device); diff: the count
    // of differing words
    uint32_t *ref = nullptr, *diff = nullptr;
    if (rc == BIGINT_OK && (hipMalloc(&ref, out_bytes) != hipSuccess ||
                            hipMalloc(&diff, sizeof(uint32_t)) != hipSuccess))
      rc = BIGINT_ENOMEM;
    bool have_ref = false;
    std::vector<uint32_t> host((size_t)nb * n);
    if (rc == BIGINT_OK) {
      uint64_t x = 0x9e3779b97f4a7c15ull ^ (uint64_t)n;  // splitmix64 stream
      auto next = [&]() {
        uint64_t z = (x += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
      };
      for (auto& v : host) v = (uint32_t)next();
      if (hipMemcpy(a, host.data(), in_bytes, hipMemcpyHostToDevice) != hipSuccess) rc = BIGINT_EHIP;
      for (auto& v : host) v = (uint32_t)next();
      if (rc == BIGINT_OK && hipMemcpy(b, host.data(), in_bytes, hipMemcpyHostToDevice) != hipSuccess)
        rc = BIGINT_EHIP;
    }
    float best = 1e30f;
    TuneEntry pick{n, 16, 8, 7};
    for (int T : kT)
    for (int D : kD)
    for (int P : kP)
      for (int W : kW) {
        if (rc != BIGINT_OK) break;
        const MfmaCfg cfg{P, W, D, T};
        // 16x16 bands: 4..16 strips; 32x32 bands: 8..32 strips, 8-bit digits,
        // a work-group per instance
        if (T == 16 && P == 32) continue;
        if (T == 32 && (D != 8 || P == 4 || W == 1)) continue;
        if (mfma_lds(n, n, cfg) > 163840) continue;
        // one wave per instance: 8-bit digits, 4 or 8 strips per band, small sizes
        if (W == 1 && (D != 8 || P == 16 || !mfma_wave_fits(n, n))) continue;
        rc = launch_mul_mfma(out, nullptr, a, n, b, n, nb, cfg, s);  // warm-up
        if (rc != BIGINT_OK) break;
        if (hipEventRecord(e0, s) != hipSuccess) { rc = BIGINT_EHIP; break; }
        for (int rep = 0; rep < 3 && rc == BIGINT_OK; ++rep)
          rc = launch_mul_mfma(out, nullptr, a, n, b, n, nb, cfg, s);
        if (rc != BIGINT_OK) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          rc = BIGINT_EHIP;
          break;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = BIGINT_EHIP; break; }
        if (!have_ref) {
          if (hipMemcpyAsync(ref, out, out_bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) {
            rc = BIGINT_EHIP;
            break;
          }
          have_ref = true;
        } else {
          uint32_t nd = 0;
          if (hipMemsetAsync(diff, 0, sizeof(uint32_t), s) != hipSuccess ||
              launch_count_diff(diff, ref, out, out_bytes / 4, s) != BIGINT_OK ||
              hipMemcpyAsync(&nd, diff, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess) {
            rc = BIGINT_EHIP;
            break;
          }
          if (nd != 0) { rc = BIGINT_EHIP; set_hip_error(hipErrorUnknown); break; }
        }
        if (ms < best) { best = ms; pick = TuneEntry{n, P, W, D, T}; }
      }
    (void)hipStreamSynchronize(s);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (out) (void)hipFree(out);
    if (ref) (void)hipFree(ref);
    if (diff) (void)hipFree(diff);
    table.push_back(pick);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  if (rc != BIGINT_OK) return rc;
  // bins switch at the geometric midpoints between the tuned sizes
  for (size_t i = 0; i + 1 < table.size(); ++i)
    table[i].max_limbs = (int)(table[i].max_limbs * 1.41421356);
  table.back().max_limbs = BIGINT_MFMA_MAX_LIMBS;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune = table;
  }
  if (cache_path) {
    FILE* f = fopen(cache_path, "w");
    if (!f) return BIGINT_EINVAL;
    int dev = 0;
    hipDeviceProp_t prop;
    (void)hipGetDevice(&dev);
    const bool have = hipGetDeviceProperties(&prop, dev) == hipSuccess;
    fprintf(f, "{\"arch\": \"%s\", \"op\": \"mul_mfma\", \"bins\": [", have ? prop.gcnArchName : "?");
    for (size_t i = 0; i < table.size(); ++i)
      fprintf(f, "%s{\"max_limbs\": %d, \"strips_per_band\": %d, \"waves\": %d, \"digit_bits\": %d, "
                 "\"tile\": %d}",
              i ? ", " : "", table[i].max_limbs, table[i].P, table[i].waves, table[i].dw, table[i].tile);
    fprintf(f, "]}\n");
    fclose(f);
  }
  return BIGINT_OK;
}

// Reads a table written by bigint_autotune (the fields are read in order);
// a null path restores the built-in table.
int bigint_autotune_load(const char* cache_path) {
  tune_env_once();
  if (!cache_path) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune = kBuiltinTune;
    return BIGINT_OK;
  }
  return load_tune_file(cache_path);
}

}  // extern "C"

namespace bi {

static int load_tune_file(const char* cache_path) {
  FILE* f = fopen(cache_path, "r");
  if (!f) return BIGINT_EINVAL;
  std::string txt;
  char buf[4096];
  size_t k;
  while ((k = fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, k);
  fclose(f);
  std::vector<TuneEntry> table;
  size_t pos = 0;
  auto field = [&](const char* name, int* v) {
    const size_t q = txt.find(name, pos);
    if (q == std::string::npos) return false;
    const size_t c = txt.find(':', q);
    if (c == std::string::npos) return false;
    // a decimal integer of int range (strtol saturates instead of overflowing)
    char* end = nullptr;
    const long x = std::strtol(txt.c_str() + c + 1, &end, 10);
    if (end == txt.c_str() + c + 1 || x < INT_MIN || x > INT_MAX) return false;
    *v = (int)x;
    pos = c + 1;
    return true;
  };
  for (;;) {
    TuneEntry e;
    if (!field("\"max_limbs\"", &e.max_limbs)) break;
    if (!field("\"strips_per_band\"", &e.P) || !field("\"waves\"", &e.waves) ||
        !field("\"digit_bits\"", &e.dw))
      return BIGINT_EINVAL;
    // "tile" (optional, 16 when absent) belongs to this entry if it comes
    // before the next entry's "max_limbs"
    {
      const size_t nt = txt.find("\"tile\"", pos), nm = txt.find("\"max_limbs\"", pos);
      if (nt != std::string::npos && (nm == std::string::npos || nt < nm) && !field("\"tile\"", &e.tile))
        return BIGINT_EINVAL;
    }
    if ((e.P != 4 && e.P != 8 && e.P != 16 && e.P != 32) ||
        (e.waves != 1 && e.waves != 4 && e.waves != 8) || (e.dw != 7 && e.dw != 8) ||
        (e.tile != 16 && e.tile != 32) || (e.P == 32 && e.tile != 32) || e.max_limbs <= 0)
      return BIGINT_EINVAL;
    table.push_back(e);
  }
  if (table.empty()) return BIGINT_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune = table;
  return BIGINT_OK;
}

}  // namespace bi
