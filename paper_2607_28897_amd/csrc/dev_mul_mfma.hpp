// dev_mul_mfma.hpp -- the MFMA-split multiply: 7-bit (or offset 8-bit)
// digits, int8 MFMA Toeplitz tiles, int32 accumulation, 64-bit recombination
// and a carry scan.
//
// What is computed is the quadratic formula of Section 5.2,
// c_k = sum_{i+j=k} alpha_i beta_j, over the 7-bit digits alpha, beta of the
// operands (digit k = bits [7k, 7k+7)), followed by a * b = sum_k c_k 2^(7k).
// Every c_k is at most min(Na, Nb) * 127^2, below 2^31 for up to 133,144
// digits, so int32 accumulation is exact with no floating point anywhere.
//
// Tiling (v_mfma_i32_16x16x64_i8, D[16x16] += A[16x64] B[64x16]):
//   A_Z[r][s] = alpha[Z + 16r - s]   (a Toeplitz slice of alpha)
//   B_Y[s][p] = beta [Y + s + p]     (overlapping windows of beta)
//   (A_Z B_Y)[r][p] = sum_{s<64} alpha[Z+16r-s] beta[Y+p+s]
// is the part of c[Z+Y+16r+p] whose beta index lies in [Y+p, Y+p+64).  With
// Z + Y = 256w fixed the 16x16 outputs are the "strip" c[256w .. 256w+256),
// and summing over all Y = 64 * integer covers every beta index once.
//   Write Y = 256y + 64rho (phase rho in 0..3) and Z = 256x - 64rho; then
// strip w = x + y.  A wave owns P consecutive strips w0..w0+P-1 (one int32
// accumulator tile each) and, per phase, walks y: strip w0+i needs A tile
// x = w0+i-y, so one step needs one new A tile and one B tile for P MFMAs;
// the other P-1 A tiles are still in registers from the previous steps (a
// ring of P tiles).  Loads per MFMA: 2/P tiles.
//
// Register layout (lane l, idx = l & 15, grp = l >> 4; operand byte t):
//   A lane holds alpha[Z + 16 idx - 16 grp - t]: 16 contiguous bytes of the
//     reversed digit array, one aligned ds_read_b128.
//   B lane holds beta[Y + idx + 16 grp + t]: 16 bytes at an offset of idx
//     bytes, assembled from 5 aligned dwords with v_alignbyte.
// Both operands use the same (grp, t) <-> contraction index map, so the
// MFMA's own K ordering inside a lane does not matter.  The result tile
// holds column p = l & 15, rows 4 (l >> 4) + v in register v.
//
// Recombination: c_k sits at bit 7k.  A strip of 256 coefficients covers
// exactly 56 limbs (7*256 = 56*32), so strips are limb-aligned.  Per strip a
// wave forms the 57 column sums X_j (lo 32 bits of every c_k 2^(7k - 32j)
// whose low bit falls in limb j, plus the high parts from limb j-1; each
// X_j < 2^35), splits X_j = L_j + 2^32 H_j, adds L + (H shifted up one
// limb) with a one-bit ballot carry scan, writes the 56 limbs and keeps the
// 57th column (with its carry) as the strip's carry word C_w.  A final
// work-group carry scan adds every C_w at limb 56(w+1).
//
// Offset 8-bit digits (DW = 8).  The digits are the bytes of the limbs
// (Na = 4 na), fed to the MFMA as alpha'_i = alpha_i - 128 in [-128, 127]
// (the byte with its top bit flipped, read as signed), zero outside [0, Na).
// Then c_k = c'_k + 128 S_k + 2^14 cnt_k with c'_k = sum alpha'_i beta'_j
// from the MFMA (|alpha' beta'| <= 2^14, so int32 is exact up to 131,071
// digits), cnt_k = the number of pairs (i, k - i) inside both operands and
// S_k = sum over those pairs of alpha'_i + beta'_{k-i}.  With PA / PB the
// prefix sums of alpha' / beta', S_k = PA(k+1) - PA(k+1-Nb) + PB(k+1) -
// PB(k+1-Na); from one k to the next it changes by alpha'_k - alpha'_{k-Nb}
// + beta'_k - beta'_{k-Na}, four digits of 4-digit groups that are limbs.
// A strip (256 coefficients = 64 limbs) takes S at its start from per-block
// (256 digit) prefix sums plus a partial block, and the rest by a wave scan
// of those differences.  The strip's limb j then takes X_j = sum_t c_{4j+t}
// 2^(8t) < 2^58, and the spill of limb 63 is the strip's carry word.
#pragma once

#include "common.hpp"
#include "dev_addsub.hpp"

namespace bi {
namespace mfma {

constexpr int kPadA = 320;  // zero bytes on both sides of reversed alpha (>= 303)
constexpr int kPadA32 = 1040;  // the same for 32x32 tiles (an A tile spans 1023 digits)
constexpr int kPadB = 64;   // zero bytes before beta (a tile reads from Y >= -64)
constexpr int kPadBt = 96;  // zero bytes after beta (reads reach Y + 80)
constexpr int kStrip = 256; // coefficients per strip

// limbs per strip of 256 coefficients: 7 * 256 / 32 and 8 * 256 / 32
template <int DW>
__host__ __device__ constexpr int strip_limbs() { return 8 * DW; }

// 7-bit digits of an n-limb integer
__host__ __device__ inline int ndigits(int n) { return (32 * n + 6) / 7; }

template <int DW>
__host__ __device__ inline int ndigits_w(int n) { return DW == 8 ? 4 * n : ndigits(n); }

struct Geo {
  int na, nb, Na, Nb;
  int QA;   // Abuf[q] = alpha[QA - q]
  int SA;   // bytes of Abuf
  int SB;   // bytes of Bbuf; Bbuf[kPadB + j] = beta[j]
  int W;    // strips
  int nout; // na + nb
  int NBa, NBb;  // 8-bit digits: 256-digit blocks of each operand
};

// nout < na + nb asks for the product mod B^nout only: the strips past limb
// nout are not computed (carries only move up, so the low limbs are exact).
// TS: the MFMA tile (16: 16x16x64, 32: 32x32x32), which sets the padding.
template <int DW, int TS = 16>
__host__ __device__ inline Geo make_geo(int na, int nb, int nout = -1) {
  constexpr int kPA = TS == 32 ? kPadA32 : kPadA;
  Geo g;
  g.na = na; g.nb = nb;
  g.Na = ndigits_w<DW>(na); g.Nb = ndigits_w<DW>(nb);
  g.NBa = (g.Na + kStrip - 1) / kStrip;
  g.NBb = (g.Nb + kStrip - 1) / kStrip;
  g.QA = ((g.Na - 1 + kPA) + 15) & ~15;
  g.SA = ((g.QA + kPA + 1) + 15) & ~15;
  g.SB = ((kPadB + g.Nb + kPadBt) + 15) & ~15;
  const int K = g.Na + g.Nb - 1;
  g.W = (K + kStrip - 1) / kStrip;
  g.nout = (nout < 0 || nout > na + nb) ? na + nb : nout;
  g.W = min(g.W, (g.nout + strip_limbs<DW>() - 1) / strip_limbs<DW>());
  return g;
}

// block prefix sums (8-bit digits): NBa + 1 and NBb + 1 ints
__host__ __device__ inline int bs_bytes(const Geo& g) { return (4 * (g.NBa + g.NBb + 2) + 15) & ~15; }

// LDS layout: [Abuf SA][Bbuf SB][per-wave scratch 1 KiB each][strip carries
// 8W][with lead (8-bit digits): every strip's limbs 0-1, 8W][band order
// 2*NB][misc 128][block prefix sums (8-bit digits)]
template <int DW, int TS = 16>
__host__ __device__ inline size_t lds_bytes(int na, int nb, int nwaves, int P, bool lead = false) {
  const Geo g = make_geo<DW, TS>(na, nb);
  const int NB = (g.W + P - 1) / P;
  return (size_t)g.SA + g.SB + (size_t)nwaves * 1024 + (size_t)((DW == 8 && lead) ? 16 : 8) * g.W +
         (size_t)((2 * NB + 15) & ~15) + 128 + (DW == 8 ? bs_bytes(g) : 0);
}

struct Lds {
  uint8_t* A;
  uint8_t* B;
  int32_t* wscr;     // this wave's 256 ints
  int32_t* scr;      // all waves' scratch (256 ints per wave)
  uint64_t* carry;   // W words
  uint64_t* lead = nullptr;  // nullable, W words: limbs 0-1 of every strip as its output wrote
                             // them, so the closing scan need not read them back from out
  uint16_t* order;   // NB entries
  uint32_t* misc;    // [0] band counter, [1..16] scan scratch (32 words)
  int32_t* bsa;      // 8-bit digits: bsa[b] = sum of alpha'_i, i < 256 b (b <= NBa)
  int32_t* bsb;      // the same for beta' (b <= NBb)
};

// lead: carve the strips' limbs 0-1 area (8-bit digits; the LDS must have
// been sized by lds_bytes with lead)
template <int DW>
__device__ __forceinline__ Lds carve(char* smem, const Geo& g, int P, bool lead) {
  Lds s;
  const int NB = (g.W + P - 1) / P;
  char* p = smem;
  s.A = reinterpret_cast<uint8_t*>(p); p += g.SA;
  s.B = reinterpret_cast<uint8_t*>(p); p += g.SB;
  s.scr = reinterpret_cast<int32_t*>(p);
  s.wscr = s.scr + wave_id() * 256; p += num_waves() * 1024;
  s.carry = reinterpret_cast<uint64_t*>(p); p += 8 * g.W;
  if (DW == 8 && lead) {
    s.lead = reinterpret_cast<uint64_t*>(p);
    p += 8 * g.W;
  }
  s.order = reinterpret_cast<uint16_t*>(p); p += (2 * NB + 15) & ~15;
  s.misc = reinterpret_cast<uint32_t*>(p); p += 128;
  s.bsa = reinterpret_cast<int32_t*>(p);
  s.bsb = s.bsa + g.NBa + 1;
  return s;
}

// Four consecutive 7-bit digits k0..k0+3 of the n-limb integer a (0 outside
// [0, 32n) bits), packed low digit first: a 28-bit window of at most two
// adjacent limbs.
__device__ __forceinline__ uint32_t digits4(const uint32_t* __restrict__ a, int n, int k0) {
  // branch-free so that the loads of consecutive calls can be batched: the
  // limb indices are clamped and the values masked instead
  const int kc = max(k0, 0);
  const int bit = 7 * kc;
  const int l = bit >> 5, sft = bit & 31;
  const uint32_t lo = a[min(l, n - 1)] & (l < n ? 0xffffffffu : 0u);
  const uint32_t hi = a[min(l + 1, n - 1)] & (l + 1 < n ? 0xffffffffu : 0u);
  const uint32_t v = (uint32_t)((((uint64_t)hi << 32) | lo) >> sft);
  const uint32_t w =
      (v & 0x7fu) | ((v << 1) & 0x7f00u) | ((v << 2) & 0x7f0000u) | ((v << 3) & 0x7f000000u);
  // k0 < 0: digits k0..-1 are padding zeros, the window at 0 moves up
  return k0 >= 0 ? w : (k0 <= -4 ? 0u : w << (8 * -k0));
}

// Limb m of an n-limb operand as four offset 8-bit digits (bytes with the
// top bit flipped: alpha' = alpha - 128 read as signed); 0 outside [0, n).
__device__ __forceinline__ uint32_t limb8(const uint32_t* __restrict__ a, int n, int m) {
  // a mask rather than a select, so that the load stays unconditional and
  // the loads of an unrolled loop issue together
  const uint32_t mask = (m >= 0 && m < n) ? 0xffffffffu : 0u;
  return (a[min(max(m, 0), n - 1)] ^ 0x80808080u) & mask;
}

// Stage the reversed digits of a and the digits of b into LDS (zero padded).
// Abuf[q] = alpha[QA - q]: dword d holds digits QA-4d-3 .. QA-4d, byte-reversed.
// (tid, T): this thread's index and the number of threads taking part
// (the whole work-group by default, one wave for the wave-level multiply)
template <int DW>
__device__ __forceinline__ void stage(const Lds& s, const Geo& g, const uint32_t* __restrict__ a,
                                      const uint32_t* __restrict__ b, int tid = -1, int T = 0) {
  if (T == 0) { tid = threadIdx.x; T = blockDim.x; }
  uint32_t* A32 = reinterpret_cast<uint32_t*>(s.A);
  uint32_t* B32 = reinterpret_cast<uint32_t*>(s.B);
  const int nA = g.SA / 4, nB = g.SB / 4;
  if constexpr (DW == 8) {
    // digits QA-4d-3 .. QA-4d: bytes 1..3 of limb l and byte 0 of limb l+1
    // (QA = 0 mod 16, so QA-4d-4 = 4l)
#pragma unroll 8
    for (int d = tid; d < nA; d += T) {
      const int l = (g.QA - 4 * d - 4) >> 2;
      const uint32_t v = __builtin_amdgcn_alignbyte(limb8(a, g.na, l + 1), limb8(a, g.na, l), 1);
      A32[d] = __builtin_bswap32(v);
    }
#pragma unroll 8
    for (int d = tid; d < nB; d += T) B32[d] = limb8(b, g.nb, d - kPadB / 4);
  } else {
#pragma unroll 8
    for (int d = tid; d < nA; d += T) {
      const int k0 = g.QA - 4 * d - 3;
      // digits at index >= Na come out 0 because the bits past the top limb are 0
      A32[d] = __builtin_bswap32(digits4(a, g.na, k0));
    }
#pragma unroll 8
    for (int d = tid; d < nB; d += T) B32[d] = digits4(b, g.nb, 4 * d - kPadB);
  }
}

// ---- 8-bit digits: sums of alpha' and beta' ---------------------------------------

// sum of the four signed digits of an offset group (0 for a zero group)
__device__ __forceinline__ int group_sum(uint32_t x) {
  return (int)__builtin_amdgcn_sad_u8(x ^ 0x80808080u, 0u, 0u) - 512;
}

// digits 4m .. 4m+3 of alpha' from the reversed buffer (byte t = digit
// 4m+3-t); 0 outside [0, na)
__device__ __forceinline__ uint32_t groupA(const uint8_t* Abuf, const Geo& g, int m) {
  const int mc = min(max(m, 0), g.na - 1);
  const uint32_t* p = reinterpret_cast<const uint32_t*>(Abuf + (g.QA - 4 * mc - 4));
  const uint32_t v = __builtin_amdgcn_alignbyte(p[1], p[0], 1);
  return v & ((m >= 0 && m < g.na) ? 0xffffffffu : 0u);
}

// digits 4m .. 4m+3 of beta' (byte t = digit 4m+t); 0 outside [0, nb)
__device__ __forceinline__ uint32_t groupB(const uint8_t* Bbuf, const Geo& g, int m) {
  const int mc = min(max(m, 0), g.nb - 1);
  const uint32_t v = reinterpret_cast<const uint32_t*>(Bbuf + kPadB)[mc];
  return v & ((m >= 0 && m < g.nb) ? 0xffffffffu : 0u);
}

// inclusive prefix sum over the 64 lanes with DPP: shifts of 1, 2, 4, 8
// inside each row of 16 lanes, then the row totals broadcast to the rows
// above (row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and 3)
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_add(int x) {
  return x + __builtin_amdgcn_update_dpp(0, x, CTRL, ROWS, 0xf, false);
}

__device__ __forceinline__ int wave_incl_scan(int x) {
  x = dpp_add<0x111, 0xf>(x);  // row_shr:1
  x = dpp_add<0x112, 0xf>(x);  // row_shr:2
  x = dpp_add<0x114, 0xf>(x);  // row_shr:4
  x = dpp_add<0x118, 0xf>(x);  // row_shr:8
  x = dpp_add<0x142, 0xa>(x);  // row_bcast:15
  x = dpp_add<0x143, 0xc>(x);  // row_bcast:31
  return x;
}

__device__ __forceinline__ int wave_sum(int x) {
  return __builtin_amdgcn_readlane(wave_incl_scan(x), 63);
}

// bsa[b] = sum of alpha'_i over i < 256 b for b = 0..NBa (bsa[NBa] is the
// whole sum); likewise bsb.  Reads the staged buffers; the caller
// synchronises before and after.
__device__ __forceinline__ void block_sums(const Lds& s, const Geo& g, int wid = -1, int nw = 0) {
  if (nw == 0) { wid = wave_id(); nw = num_waves(); }
  // a row of 16 lanes per block, four consecutive groups per lane (no LDS
  // bank conflicts); the row total by DPP shifts inside the row
  const int nblk = g.NBa + g.NBb;
  const int lane = lane_id(), row = lane >> 4, col = lane & 15;
  for (int t0 = 4 * wid; t0 < nblk; t0 += 4 * nw) {
    const int t = t0 + row;
    const bool isA = t < g.NBa;
    const int blk = isA ? t : t - g.NBa;
    const int m = 64 * blk + 4 * col;
    int v = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) v += group_sum(isA ? groupA(s.A, g, m + e) : groupB(s.B, g, m + e));
    v = dpp_add<0x111, 0xf>(v);  // row_shr:1
    v = dpp_add<0x112, 0xf>(v);  // row_shr:2
    v = dpp_add<0x114, 0xf>(v);  // row_shr:4
    v = dpp_add<0x118, 0xf>(v);  // row_shr:8
    if (col == 15 && t < nblk) (isA ? s.bsa : s.bsb)[blk + 1] = v;
  }
}

// exclusive prefix over the block totals (wave 0: alpha', wave 1 or 0: beta')
__device__ __forceinline__ void block_prefix(const Lds& s, const Geo& g, int wid = -1, int nw = 0) {
  if (nw == 0) { wid = wave_id(); nw = num_waves(); }
  for (int op = 0; op < 2; ++op) {
    if (wid != (nw > 1 ? op : 0)) continue;
    int32_t* bs = op == 0 ? s.bsa : s.bsb;
    const int nb = op == 0 ? g.NBa : g.NBb;
    int carry = 0;
    for (int base = 0; base < nb; base += 64) {
      const int b = base + lane_id();
      const int v = b < nb ? bs[b + 1] : 0;
      const int inc = wave_incl_scan(v) + carry;
      if (b < nb) bs[b + 1] = inc;
      carry = __builtin_amdgcn_readlane(inc, 63);
    }
    if (lane_id() == 0) bs[0] = 0;
  }
}

// prefix sum of alpha' (or beta') over digits [0, 4 gx) = a block prefix
// (the whole blocks below gx, returned in .base, the same in every lane)
// plus this lane's group of the partial block when it lies below gx (.part;
// the wave-wide sum of .part completes it).
struct Prefix { int base, part; };

__device__ __forceinline__ Prefix prefix_groups(const Lds& s, const Geo& g, bool isA, int gx) {
  const int n = isA ? g.na : g.nb;
  const int32_t* bs = isA ? s.bsa : s.bsb;
  const int gc = min(max(gx, 0), n);
  const int blk = gc >> 6;
  const int m = 64 * blk + lane_id();
  const uint32_t x = m < gc ? (isA ? groupA(s.A, g, m) : groupB(s.B, g, m)) : 0u;
  return Prefix{bs[blk], group_sum(x)};
}

// y range of phase rho for the band starting at strip w0 (P strips).
struct Range { int lo, hi, xlo, xhi; };

__device__ __forceinline__ Range band_range(const Geo& g, int w0, int P, int rho) {
  Range r;
  // B tile covers beta[Y .. Y+78]; it is nonzero iff that meets [0, Nb)
  const int yb_lo = ceil_div(-78 - 64 * rho, 256);
  const int yb_hi = floor_div(g.Nb - 1 - 64 * rho, 256);
  // A tile covers alpha[Z-63 .. Z+240]; nonzero iff that meets [0, Na)
  r.xlo = ceil_div(64 * rho - 240, 256);
  r.xhi = floor_div(g.Na + 62 + 64 * rho, 256);
  r.lo = max(yb_lo, w0 - r.xhi);
  r.hi = min(yb_hi, w0 + P - 1 - r.xlo);
  return r;
}

__device__ __forceinline__ int band_cost(const Geo& g, int band, int P) {
  int c = 0;
  for (int rho = 0; rho < 4; ++rho) {
    const Range r = band_range(g, band * P, P, rho);
    c += max(0, r.hi - r.lo + 1);
  }
  return c;
}

// A tile x of phase rho.  Tiles entirely outside alpha read the zero padding
// at the start of Abuf (every lane the same 16 bytes), so no branch is needed.
__device__ __forceinline__ v4i load_A(const uint8_t* Abuf, const Geo& g, int x, int rho,
                                      const Range& r) {
  const int lane = lane_id();
  const int Z = 256 * x - 64 * rho;
  const bool ok = x >= r.xlo && x <= r.xhi;  // wave-uniform
  const int addr = ok ? g.QA - Z - 16 * (lane & 15) + 16 * (lane >> 4) : 0;
  return *reinterpret_cast<const v4i*>(Abuf + addr);
}

// B tile y of phase rho in two halves: the five aligned dwords a lane needs
// (issued early) and their byte alignment into the operand (done late).
struct BRaw {
  uint32_t d[5];
};

__device__ __forceinline__ BRaw load_B_raw(const uint8_t* Bbuf, int y, int rho) {
  const int lane = lane_id();
  const int p = lane & 15;
  const int Y = 256 * y + 64 * rho;
  const uint32_t* src =
      reinterpret_cast<const uint32_t*>(Bbuf + kPadB + Y + 16 * (lane >> 4) + 4 * (p >> 2));
  BRaw b;
#pragma unroll
  for (int i = 0; i < 5; ++i) b.d[i] = src[i];
  return b;
}

__device__ __forceinline__ v4i align_B(const BRaw& b) {
  const uint32_t sh = lane_id() & 3;
  v4i v;
  v.x = (int)__builtin_amdgcn_alignbyte(b.d[1], b.d[0], sh);
  v.y = (int)__builtin_amdgcn_alignbyte(b.d[2], b.d[1], sh);
  v.z = (int)__builtin_amdgcn_alignbyte(b.d[3], b.d[2], sh);
  v.w = (int)__builtin_amdgcn_alignbyte(b.d[4], b.d[3], sh);
  return v;
}

// One phase of one band: acc[i] += sum over the y range of A(w0+i-y) B(y).
// Software pipeline per step: the step's P MFMAs run on the B tile aligned at
// the end of the previous step; the raw dwords of the next B tile were loaded
// one step earlier, and the one new A tile goes into the ring slot that the
// first MFMA of the step has just read.
//
// Band edges: where the low end of the band's y range is set by the A
// operand (the upper half of the product), strip i's first useful step is i,
// so the first P-1 steps hold a staircase of MFMAs on all-zero A tiles.
// There the first P steps run as a "ramp" block that leaves those MFMAs out
// at compile time.  (The mirror staircase at the high end of the range, in
// the lower half of the product, is kept: walking those ranges downwards
// with reversed accumulators measured slower, its extra registers costing
// more than the MFMAs it saves.)
template <int P>
__device__ __forceinline__ void band_phase(v4i (&acc)[P], const Lds& s, const Geo& g, int w0,
                                           int rho) {
  const Range r = band_range(g, w0, P, rho);
  const int L = r.hi - r.lo + 1;
  if (L <= 0) return;
  const int xb = w0 - r.lo;  // strip i at step u uses x = xb + i - u
  // the low end of the range is set by the A operand: strip i starts at step i
  const bool ramp = L >= 2 * P && r.lo == w0 - r.xhi;
  v4i ring[P];
#pragma unroll
  for (int i = 0; i < P; ++i) ring[i] = load_A(s.A, g, xb + i, rho, r);
  v4i Bc = align_B(load_B_raw(s.B, r.lo, rho));
  BRaw raw = load_B_raw(s.B, min(r.lo + 1, r.hi), rho);

  // one step (st = step mod P and the ramp flag known at compile time).  The
  // next B tile is aligned into a second register set half-way through the
  // step, so the step boundary carries no VALU -> MFMA dependency.
  auto step_fn = [&](const int step, const int st, const bool rmp) __attribute__((always_inline)) {
    auto mma = [&](int i) __attribute__((always_inline)) {
      if (!rmp || i <= st)
        acc[i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ring[(P + i - st) % P], Bc, acc[i], 0, 0, 0);
    };
    // strip P-1 first: its slot is the one the next step's new tile takes
    mma(P - 1);
    ring[(2 * P - 1 - st) % P] = load_A(s.A, g, xb - step - 1, rho, r);
#pragma unroll
    for (int i = P - 2; i >= P / 2; --i) mma(i);
    __builtin_amdgcn_sched_barrier(0);
    const v4i Bn = align_B(raw);
    raw = load_B_raw(s.B, min(r.lo + step + 2, r.hi), rho);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = P / 2 - 1; i >= 0; --i) mma(i);
    __builtin_amdgcn_sched_barrier(0);
    Bc = Bn;
  };
  // full blocks of P steps: no exit inside, the ring returns to its layout
  const int nfull = L / P;
  int blk0 = 0;
  if (ramp) {
#pragma unroll
    for (int st = 0; st < P; ++st) step_fn(st, st, true);
    blk0 = 1;
  }
#pragma unroll 1
  for (int blk = blk0; blk < nfull; ++blk) {
#pragma unroll
    for (int st = 0; st < P; ++st) step_fn(blk * P + st, st, false);
  }
  // the remaining L mod P steps
  const int rem = L - nfull * P;
  if (rem > 0) {
    // a guarded, fully unrolled block keeps every ring index a constant
#pragma unroll
    for (int st = 0; st < P - 1; ++st)
      if (st < rem) step_fn(nfull * P + st, st, false);
  }
}

// Per strip: turn the 256 coefficients of acc (strip w) into 56 limbs of out
// and the strip carry word; or, for the diagnostic path, store them raw.
__device__ __forceinline__ void strip_out7(v4i acc, int w, const Lds& s, const Geo& g,
                                           uint32_t* out, int32_t* coef) {
  constexpr int kStripLimbs = strip_limbs<7>();
  const int lane = lane_id();
  int32_t* sc = s.wscr;
  // lane l holds column p = l & 15, rows 4(l>>4)+v: coefficient 16 row + p
#pragma unroll
  for (int v = 0; v < 4; ++v) sc[16 * (4 * (lane >> 4) + v) + (lane & 15)] = acc[v];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (coef) {
    const int K = g.Na + g.Nb - 1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int kk = 64 * v + lane;
      const int k = kStrip * w + kk;
      if (k < K) coef[k] = sc[kk];
    }
    __builtin_amdgcn_wave_barrier();
    return;
  }
  // column sums: lane j in [0, 57) gathers the coefficients of limb j (at
  // most 5 whose low bits start in limb j, at most 5 spilling from limb j-1);
  // fixed trip counts with masks keep the LDS reads unconditional
  uint64_t X = 0;
  {
    const int j = min(lane, kStripLimbs);
    const int klo = (32 * j + 6) / 7;          // first kappa with floor(7 kappa/32) == j
    const int khi = (32 * (j + 1) + 6) / 7;    // one past the last
    const int plo = (32 * (j - 1) + 6) / 7;    // first kappa of limb j-1 (j > 0)
#pragma unroll
    for (int e = 0; e < 5; ++e) {
      const int kk = klo + e;
      const uint64_t v = (uint64_t)(uint32_t)sc[min(kk, kStrip - 1)] << ((7 * kk - 32 * j) & 63);
      X += (kk < khi && kk < kStrip) ? (v & 0xffffffffull) : 0ull;
      const int pk = plo + e;
      const uint64_t u = (uint64_t)(uint32_t)sc[max(min(pk, kStrip - 1), 0)]
                         << ((7 * pk - 32 * (j - 1)) & 63);
      X += (j > 0 && pk < klo) ? (u >> 32) : 0ull;
    }
    if (lane > kStripLimbs) X = 0;
  }
  __builtin_amdgcn_wave_barrier();
  const uint32_t L = (uint32_t)X;
  const uint32_t H = (uint32_t)(X >> 32);
  // H of the lane below, 0 into lane 0 (DPP wave_shr:1)
  const uint32_t Hprev = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)H, 0x138, 0xf, 0xf, false);
  const uint64_t sum = (uint64_t)L + Hprev;
  const uint32_t res = (uint32_t)sum;
  const bool gb = (sum >> 32) != 0;
  const bool pb = (lane <= kStripLimbs) && res == 0xffffffffu;
  const WaveCarry wc = wave_carry_masks(gb, pb);
  const uint32_t cin = wave_carry_in(wc, 0);
  const uint32_t limb = res + cin;
  const int jg = kStripLimbs * w + lane;
  // limbs 2..55 all ones (limbs past the product count as ones): a carry
  // entering limb 2 then runs through the whole strip
  const uint64_t tail = ((1ull << kStripLimbs) - 1) & ~3ull;
  const uint64_t ones = __ballot(jg >= g.nout || limb == 0xffffffffu);
  if (lane < kStripLimbs) {
    if (jg < g.nout) out[jg] = limb;
  } else if (lane == kStripLimbs) {
    const uint32_t cout = (uint32_t)gb | ((uint32_t)pb & cin);
    s.carry[w] = (uint64_t)limb | ((uint64_t)(H + cout) << 32) |
                 ((uint64_t)((ones & tail) == tail) << 63);
  }
}

// The same for offset 8-bit digits: the strip's 64 limbs and its carry word.
// S_{256w-1} = PA(256w) - PA(256w-Nb) + PB(256w) - PB(256w-Na), the digit-sum
// term at the start of strip w: block prefixes, plus a partial block where a
// boundary is not block-aligned (the tests are wave-uniform).  Later strips of
// a band carry it forward instead (strip_out8 returns the next one).
__device__ __forceinline__ int strip_start_sum(const Lds& s, const Geo& g, int w) {
  const int lane = lane_id();
  const int g0 = 64 * w;
  int S0 = 0, part = 0;
  bool partial = false;
  auto pre = [&](bool isA, int gx, int sign) __attribute__((always_inline)) {
    const int n = isA ? g.na : g.nb;
    const int gc = min(max(gx, 0), n);
    const int blk = gc >> 6;
    S0 += sign * (isA ? s.bsa : s.bsb)[blk];
    if (gc & 63) {
      partial = true;
      const int m = 64 * blk + lane;
      const uint32_t x = m < gc ? (isA ? groupA(s.A, g, m) : groupB(s.B, g, m)) : 0u;
      part += sign * group_sum(x);
    }
  };
  pre(true, g0, 1);
  pre(true, g0 - g.nb, -1);
  pre(false, g0, 1);
  pre(false, g0 - g.na, -1);
  if (partial) S0 += wave_sum(part);
  return S0;
}

// Strip w with offset 8-bit digits: its 64 limbs and carry word.  S0 is the
// digit-sum term at the strip start; returns the one of strip w + 1.
// TS = 32: acc is a quarter of a 32x32 result tile (registers 4q..4q+3:
// column lane & 31, rows 4 (lane >> 5) + v of the quarter's eight).
template <int TS = 16>
__device__ __forceinline__ int strip_out8(v4i acc, int w, const Lds& s, const Geo& g,
                                          uint32_t* out, int S0) {
  const int lane = lane_id();
  int32_t* sc = s.wscr;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if constexpr (TS == 32) sc[32 * (4 * (lane >> 5) + v) + (lane & 31)] = acc[v];
    else sc[16 * (4 * (lane >> 4) + v) + (lane & 15)] = acc[v];
  }
  const int g0 = 64 * w;         // the strip's first limb (4-digit group)
  const int m1 = g0 + lane;      // this lane's limb; its digits k = 4 m1 + t
  // per-digit changes of S: alpha'_k - alpha'_{k-Nb} + beta'_k - beta'_{k-Na};
  // a group range entirely outside its operand is skipped (wave-uniform)
  int d[4] = {0, 0, 0, 0};
  int sigma = 0;
  auto add_group = [&](uint32_t x, int sign, bool rev) __attribute__((always_inline)) {
    sigma += sign * group_sum(x);
#pragma unroll
    for (int t = 0; t < 4; ++t) d[t] += sign * __builtin_amdgcn_sbfe((int)x, 8 * (rev ? 3 - t : t), 8);
  };
  auto live = [&](int lo, int n) { return lo + 63 >= 0 && lo < n; };  // [lo, lo+64) meets [0, n)
  if (live(g0, g.na)) add_group(groupA(s.A, g, m1), 1, true);
  if (live(g0 - g.nb, g.na)) add_group(groupA(s.A, g, m1 - g.nb), -1, true);
  if (live(g0, g.nb)) add_group(groupB(s.B, g, m1), 1, false);
  if (live(g0 - g.na, g.nb)) add_group(groupB(s.B, g, m1 - g.na), -1, false);
  const int incl = wave_incl_scan(sigma);
  const int excl = incl - sigma;
  const int S_next = S0 + __builtin_amdgcn_readlane(incl, 63);
  // pair counts cnt_k = min(k+1, Na) - max(0, k+1-Nb) (clamped at 0) change by
  // the same step for the four digits of a limb: both bounds are multiples of 4
  const int k0 = 4 * m1;
  const int cnt0 = min(k0 + 1, g.Na) - max(0, k0 + 1 - g.Nb);
  const int step = (k0 + 4 <= g.Na ? 1 : 0) - (m1 >= g.nb ? 1 : 0);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const v4i cp = *reinterpret_cast<const v4i*>(sc + 4 * lane);
  int S = S0 + excl;
  uint64_t X = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    S += d[t];
    const int cnt = max(0, cnt0 + t * step);
    // c_k = c'_k + 128 (S_k + 128 cnt_k), at most 2^33
    const int64_t c = (int64_t)cp[t] + ((int64_t)(S + 128 * cnt) << 7);
    X += (uint64_t)c << (8 * t);
  }
  __builtin_amdgcn_wave_barrier();
  const uint32_t L = (uint32_t)X;
  const uint32_t H = (uint32_t)(X >> 32);
  // H of the lane below, 0 into lane 0 (DPP wave_shr:1)
  const uint32_t Hprev = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)H, 0x138, 0xf, 0xf, false);
  const uint64_t sum = (uint64_t)L + Hprev;
  const uint32_t res = (uint32_t)sum;
  const bool gb = (sum >> 32) != 0;
  const bool pb = res == 0xffffffffu;
  const WaveCarry wc = wave_carry_masks(gb, pb);
  const uint32_t cin = wave_carry_in(wc, 0);
  const uint32_t limb = res + cin;
  const int jg = g0 + lane;
  const uint64_t tail = ~3ull;   // limbs 2..63
  const uint64_t ones = __ballot(jg >= g.nout || limb == 0xffffffffu);
  if (jg < g.nout) out[jg] = limb;
  if (s.lead && lane < 2) reinterpret_cast<uint32_t*>(s.lead)[2 * w + lane] = jg < g.nout ? limb : 0u;
  if (lane == 63) {
    const uint32_t cout = (uint32_t)gb | ((uint32_t)pb & cin);
    s.carry[w] = (uint64_t)(H + cout) | ((uint64_t)((ones & tail) == tail) << 63);
  }
  return S_next;
}

// ---- 32x32x32 tiles (v_mfma_i32_32x32x32_i8) ----------------------------------------
// D[32x32] += A[32x32] B[32x32] with A_Z[r][s] = alpha[Z + 32r - s] and
// B_Y[s][p] = beta[Y + s + p]: the 1024 outputs are c[Z+Y .. Z+Y+1024),
// tile T = four consecutive strips.  With Y = 1024y + 32rho (32 phases) and
// Z = 1024x - 32rho the tile is T = x + y, and a band of P/4 tiles walks y
// with a ring of A tiles exactly as the 16x16 bands do.  Each instruction
// does twice the 16x16x64 tile's multiply-accumulates for the same operand
// bytes per lane.  Register layout (lane l, row r = l & 31, k-group
// g = l >> 5, byte t: contraction index 16g + t): A lane holds
// alpha[Z + 32r - 16g - t], one aligned ds_read_b128 of the reversed
// digits; B lane holds beta[Y + p + 16g + t] with p = l & 31, five dwords
// aligned with v_alignbyte.  Result register v holds column l & 31, row
// (v & 3) + 8 (v >> 2) + 4 (l >> 5): registers 4q..4q+3 are strip 4T + q.
typedef int v16i __attribute__((ext_vector_type(16)));

__device__ __forceinline__ Range band_range32(const Geo& g, int T0, int P32, int rho) {
  Range r;
  // B tile covers beta[Y .. Y+62]; A tile covers alpha[Z-31 .. Z+992]
  const int yb_lo = ceil_div(-62 - 32 * rho, 1024);
  const int yb_hi = floor_div(g.Nb - 1 - 32 * rho, 1024);
  r.xlo = ceil_div(32 * rho - 992, 1024);
  r.xhi = floor_div(g.Na + 30 + 32 * rho, 1024);
  r.lo = max(yb_lo, T0 - r.xhi);
  r.hi = min(yb_hi, T0 + P32 - 1 - r.xlo);
  return r;
}

__device__ __forceinline__ int band_cost32(const Geo& g, int band, int P) {
  int c = 0;
  for (int rho = 0; rho < 32; ++rho) {
    const Range r = band_range32(g, band * (P / 4), P / 4, rho);
    c += max(0, r.hi - r.lo + 1);
  }
  return c;
}

__device__ __forceinline__ v4i load_A32(const uint8_t* Abuf, const Geo& g, int x, int rho,
                                        const Range& r) {
  const int lane = lane_id();
  const int Z = 1024 * x - 32 * rho;
  const bool ok = x >= r.xlo && x <= r.xhi;  // wave-uniform
  const int addr = ok ? g.QA - Z - 32 * (lane & 31) + 16 * (lane >> 5) : 0;
  return *reinterpret_cast<const v4i*>(Abuf + addr);
}

__device__ __forceinline__ BRaw load_B_raw32(const uint8_t* Bbuf, int y, int rho) {
  const int lane = lane_id();
  const int p = lane & 31;
  const int Y = 1024 * y + 32 * rho;
  const uint32_t* src =
      reinterpret_cast<const uint32_t*>(Bbuf + kPadB + Y + 16 * (lane >> 5) + 4 * (p >> 2));
  BRaw b;
#pragma unroll
  for (int i = 0; i < 5; ++i) b.d[i] = src[i];
  return b;
}

// One phase of one band of P32 tiles: acc[i] += sum over the y range of
// A(T0+i-y) B(y); the software pipeline and the ramp block of band_phase.
template <int P32>
__device__ __forceinline__ void band_phase32(v16i (&acc)[P32], const Lds& s, const Geo& g, int T0,
                                             int rho) {
  const Range r = band_range32(g, T0, P32, rho);
  const int L = r.hi - r.lo + 1;
  if (L <= 0) return;
  const int xb = T0 - r.lo;
  const bool ramp = L >= 2 * P32 && r.lo == T0 - r.xhi;
  v4i ring[P32];
#pragma unroll
  for (int i = 0; i < P32; ++i) ring[i] = load_A32(s.A, g, xb + i, rho, r);
  v4i Bc = align_B(load_B_raw32(s.B, r.lo, rho));
  BRaw raw = load_B_raw32(s.B, min(r.lo + 1, r.hi), rho);
  auto step_fn = [&](const int step, const int st, const bool rmp) __attribute__((always_inline)) {
    auto mma = [&](int i) __attribute__((always_inline)) {
      if (!rmp || i <= st)
        acc[i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ring[(P32 + i - st) % P32], Bc, acc[i], 0, 0, 0);
    };
    mma(P32 - 1);
    ring[(2 * P32 - 1 - st) % P32] = load_A32(s.A, g, xb - step - 1, rho, r);
#pragma unroll
    for (int i = P32 - 2; i >= P32 / 2; --i) mma(i);
    __builtin_amdgcn_sched_barrier(0);
    const v4i Bn = align_B(raw);
    raw = load_B_raw32(s.B, min(r.lo + step + 2, r.hi), rho);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = P32 / 2 - 1; i >= 0; --i) mma(i);
    __builtin_amdgcn_sched_barrier(0);
    Bc = Bn;
  };
  const int nfull = L / P32;
  int blk0 = 0;
  if (ramp) {
#pragma unroll
    for (int st = 0; st < P32; ++st) step_fn(st, st, true);
    blk0 = 1;
  }
#pragma unroll 1
  for (int blk = blk0; blk < nfull; ++blk) {
#pragma unroll
    for (int st = 0; st < P32; ++st) step_fn(blk * P32 + st, st, false);
  }
  const int rem = L - nfull * P32;
  if (rem > 0) {
#pragma unroll
    for (int st = 0; st < P32 - 1; ++st)
      if (st < rem) step_fn(nfull * P32 + st, st, false);
  }
}

// A band of P strips (P / 4 tiles of 32x32) with offset 8-bit digits.
template <int P>
__device__ __forceinline__ void run_band32(int band, const Lds& s, const Geo& g, uint32_t* out) {
  constexpr int P32 = P / 4;
  const int T0 = band * P32;
  v16i acc[P32];
#pragma unroll
  for (int i = 0; i < P32; ++i) {
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[i][e] = 0;
  }
#pragma unroll 1
  for (int rho = 0; rho < 32; ++rho) band_phase32<P32>(acc, s, g, T0, rho);
  int S = 0;
#pragma unroll
  for (int i = 0; i < P32; ++i) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int w = 4 * (T0 + i) + q;
      if (w < g.W) {
        if (i == 0 && q == 0) S = strip_start_sum(s, g, w);
        const v4i part = {acc[i][4 * q], acc[i][4 * q + 1], acc[i][4 * q + 2], acc[i][4 * q + 3]};
        S = strip_out8<32>(part, w, s, g, out, S);
      }
    }
  }
}

template <int DW, int P>
__device__ __forceinline__ void run_band(int band, const Lds& s, const Geo& g, uint32_t* out, int32_t* coef) {
  const int w0 = band * P;
  v4i acc[P];
#pragma unroll
  for (int i = 0; i < P; ++i) acc[i] = v4i{0, 0, 0, 0};
#pragma unroll 1
  for (int rho = 0; rho < 4; ++rho) band_phase<P>(acc, s, g, w0, rho);
  int S = 0;
#pragma unroll
  for (int i = 0; i < P; ++i)
    if (w0 + i < g.W) {
      if constexpr (DW == 8) {
        if (i == 0) S = strip_start_sum(s, g, w0);
        S = strip_out8(acc[i], w0 + i, s, g, out, S);
      } else {
        strip_out7(acc[i], w0 + i, s, g, out, coef);
      }
    }
}

// The closing strip carry scan of an instance (whole work-group): carry[w]
// holds strip w's carry word (bits 0-62) and tail flag (bit 63), out its
// limbs, strips from w_first up; scratch: >= 16 words of LDS.  lead
// (nullable, LDS): lead[w] = strip w's limbs 0-1 as written to out, read
// there instead of from out.
template <int DW>
__device__ __forceinline__ void close_strips(uint32_t* out, const Geo& g, const uint64_t* carry, int w_first,
                                             uint32_t* scratch, const uint64_t* lead = nullptr) {
  constexpr int kStripLimbs = strip_limbs<DW>();
  // out += sum_w C_w B^(L(w+1)), L limbs per strip.  Strip w' receives C_{w'-1} (< 2^35) on its
  // limbs 0 and 1; a carry out of limb 1 runs on only through a tail of
  // all-ones limbs.  So an exclusive carry scan over strips, one strip per
  // thread, resolves everything: strip w' generates when limbs 0..1 plus
  // C_{w'-1} overflow and its tail is all ones, and propagates when limbs
  // 0..1 plus C_{w'-1} are all ones and so is its tail.
  const uint64_t kC = (1ull << 63) - 1;
  uint32_t cy = 0u;
  for (int base = w_first; base < g.W; base += blockDim.x) {
    const int w = base + threadIdx.x;
    const bool valid = w < g.W;
    const int j0 = kStripLimbs * (valid ? w : 0);
    uint64_t x0;
    if (lead) {
      x0 = valid ? lead[w] : 0ull;
    } else {
      const uint32_t l0 = (valid && j0 < g.nout) ? out[j0] : 0u;
      const uint32_t l1 = (valid && j0 + 1 < g.nout) ? out[j0 + 1] : 0u;
      x0 = ((uint64_t)l1 << 32) | l0;
    }
    const uint64_t d = (valid && w > w_first) ? (carry[w - 1] & kC) : 0ull;
    const bool ones = valid && (carry[w] >> 63);
    const uint64_t x = x0 + d;
    const bool xh = x < x0;  // carry out of limb 1
    const bool gen = valid && xh && ones;
    const bool prop = valid && !xh && x == ~0ull && ones;
    uint32_t cout;
    const uint32_t c = wg_carry_scan(gen, prop, cy, scratch, &cout);
    cy = cout;
    if (valid) {
      const uint64_t y = x + c;
      const bool yh = xh || (y < x);
      if (y != x0) {
        if (j0 < g.nout) out[j0] = (uint32_t)y;
        if (j0 + 1 < g.nout) out[j0 + 1] = (uint32_t)(y >> 32);
      }
      if (yh) {  // ripple into the tail (stops at its first limb that is not all ones)
        for (int j = j0 + 2; j < min(j0 + kStripLimbs, g.nout); ++j) {
          const uint32_t v = out[j];
          out[j] = v + 1u;
          if (v != 0xffffffffu) break;
        }
      }
    }
  }
}

// First band of a product whose limbs below nlo are not needed: the strips
// of the bands before it lie entirely below limb nlo - 2.  (The part of the
// product they hold is below 2^34 B^(first strip's limb) <= B^nlo, so leaving
// it out lowers floor(a b / B^nlo) by at most one.)
template <int DW>
__host__ __device__ inline int high_band(int nlo, int P) {
  return nlo > 2 ? ((nlo - 2) / strip_limbs<DW>()) / P : 0;
}

// out[0 .. nout) = a * b mod B^nout for one instance (whole work-group),
// digits of DW bits; nout < 0 means the whole na+nb limbs.  nlo > 0 asks
// only for the limbs from nlo up: the bands below high_band(nlo) are not
// computed, out[nlo ..) then holds floor(a b / B^nlo) mod B^(nout-nlo) or
// one less, and the limbs below nlo are left as they were or wrong.  With
// coef != nullptr (7-bit digits only, whole product) the raw coefficients
// c_k (k < Na+Nb-1) are written instead.
// nparts > 1 (full products, coef == nullptr, nlo == 0): this work-group is
// part `part` of nparts sharing the instance.  The bands are cut into nparts
// contiguous runs of about equal cost (band t goes to the part its cost
// midpoint falls in); this part computes only its run, writes its strips'
// carry words to carry_ext[w] (global memory, one word per strip) instead of
// LDS and leaves the closing strip carry scan to close_strips once every
// part has finished (a later launch).
// lead (8-bit digits, whole instance; smem sized by lds_bytes with lead):
// every strip's limbs 0-1 are also kept in LDS, where the closing scan reads
// them instead of reading them back from out.
template <int DW, int P, int TS = 16>
__device__ __forceinline__ void wg_mul_mfma(uint32_t* out, int32_t* coef, const uint32_t* __restrict__ a, int na,
                            const uint32_t* __restrict__ b, int nb, char* smem, int nout = -1,
                            int nlo = 0, int part = 0, int nparts = 1, uint64_t* carry_ext = nullptr,
                            bool lead = false) {
  static_assert(DW == 7 || DW == 8, "digit width");
  static_assert(TS == 16 || (TS == 32 && DW == 8 && P % 4 == 0), "32x32 tiles: 8-bit digits, whole tiles per band");
  const Geo g = make_geo<DW, TS>(na, nb, coef ? -1 : nout);
  Lds s = carve<DW>(smem, g, P, lead && coef == nullptr && nparts == 1);
  if (nparts > 1) s.carry = carry_ext;
  const int NBall = (g.W + P - 1) / P;
  // bands [band_lo, NBall) are computed; strips from w_first up
  const int band_lo = coef ? 0 : min(high_band<DW>(nlo, P), NBall);
  const int w_first = band_lo * P;
  const int NB = NBall - band_lo;

  stage<DW>(s, g, a, b);
  if constexpr (DW == 8) {
    __syncthreads();
    block_sums(s, g);
    __syncthreads();
    block_prefix(s, g);
  }
  // band order: most expensive first (rank sort by cost; the costs sit in
  // the wave scratch area, which holds 256 ints per wave >= NB)
  for (int t = threadIdx.x; t < NB; t += blockDim.x)
    s.scr[t] = TS == 32 ? band_cost32(g, band_lo + t, P) : band_cost(g, band_lo + t, P);
  if (threadIdx.x == 0) s.misc[0] = 0;
  __syncthreads();
  // this part's bands [pb0, pb1) (all of them for a whole instance)
  int pb0 = 0, pb1 = NB;
  if (nparts > 1) {
    if (threadIdx.x == 0) {
      int64_t tot = 0;
      for (int t = 0; t < NB; ++t) tot += s.scr[t];
      int64_t acc = 0;
      int b0 = NB, b1 = NB;
      for (int t = 0; t < NB; ++t) {
        const int64_t c2 = 2 * acc + s.scr[t];   // twice the cost midpoint
        const int pt = tot > 0 ? (int)min<int64_t>(nparts - 1, c2 * nparts / (2 * tot)) : 0;
        if (pt >= part && b0 == NB) b0 = t;
        if (pt > part && b1 == NB) b1 = t;
        acc += s.scr[t];
      }
      s.misc[1] = (uint32_t)b0;
      s.misc[2] = (uint32_t)max(b0, b1);
    }
    __syncthreads();
    pb0 = (int)s.misc[1];
    pb1 = (int)s.misc[2];
  }
  const int PN = pb1 - pb0;
  for (int t = threadIdx.x; t < PN; t += blockDim.x) {
    const int c = s.scr[pb0 + t];
    int rank = 0;
    for (int u2 = 0; u2 < PN; ++u2) {
      const int cu = s.scr[pb0 + u2];
      rank += (cu > c) || (cu == c && u2 < t);
    }
    s.order[rank] = (uint16_t)(pb0 + t);
  }
  __syncthreads();

  for (;;) {
    uint32_t t = 0;
    if (lane_id() == 0) t = atomicAdd(&s.misc[0], 1u);
    t = __builtin_amdgcn_readfirstlane(t);
    if ((int)t >= PN) break;
    const int band = band_lo + __builtin_amdgcn_readfirstlane((int)s.order[t]);
    if constexpr (TS == 32) run_band32<P>(band, s, g, out);
    else run_band<DW, P>(band, s, g, out, coef);
  }
  __syncthreads();
  if (coef == nullptr && nparts == 1) close_strips<DW>(out, g, s.carry, w_first, s.misc + 1, s.lead);
  __syncthreads();
}

// ---- one wave per instance (small operands) ----------------------------------------
// For operands of a few hundred limbs the work-group phases (staging, block
// sums, band scheduling, the strip carry scan) and their barriers cost more
// than the MFMA work, so several instances share a work-group, one wave each
// (the paper's ipb instances per block), and every phase runs inside the
// wave: the same staging, block sums and bands, and the strip carry scan on
// one lane per strip.  Needs W <= 64 strips (na + nb <= 4096 limbs).

// LDS bytes of one wave's instance (8-bit digits): operands, the wave's
// scratch, strip carries, misc, block prefix sums
__host__ __device__ inline size_t wave_lds_bytes(int na, int nb) {
  const Geo g = make_geo<8>(na, nb);
  return (((size_t)g.SA + g.SB + 1024 + (size_t)8 * g.W + 128 + bs_bytes(g)) + 15) & ~(size_t)15;
}

__device__ __forceinline__ Lds carve_wave(char* smem, const Geo& g) {
  Lds s;
  char* p = smem;
  s.A = reinterpret_cast<uint8_t*>(p); p += g.SA;
  s.B = reinterpret_cast<uint8_t*>(p); p += g.SB;
  s.scr = s.wscr = reinterpret_cast<int32_t*>(p); p += 1024;
  s.carry = reinterpret_cast<uint64_t*>(p); p += 8 * g.W;
  s.order = nullptr;
  s.misc = reinterpret_cast<uint32_t*>(p); p += 128;
  s.bsa = reinterpret_cast<int32_t*>(p);
  s.bsb = s.bsa + g.NBa + 1;
  return s;
}

// LDS writes of this wave visible to its later LDS reads
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// out[0 .. nout) = a * b mod B^nout on the calling wave alone (offset 8-bit
// digits; nout < 0: the whole na+nb limbs); smem: wave_lds_bytes(na, nb)
// bytes of this wave's own LDS.
template <int P>
__device__ __forceinline__ void wave_mul_mfma(uint32_t* out, const uint32_t* __restrict__ a, int na,
                                              const uint32_t* __restrict__ b, int nb, char* smem,
                                              int nout = -1) {
  const Geo g = make_geo<8>(na, nb, nout);
  const Lds s = carve_wave(smem, g);
  const int lane = lane_id();
  stage<8>(s, g, a, b, lane, 64);
  wave_sync();
  block_sums(s, g, 0, 1);
  wave_sync();
  block_prefix(s, g, 0, 1);
  wave_sync();
  const int NB = (g.W + P - 1) / P;
#pragma unroll 1
  for (int band = 0; band < NB; ++band) run_band<8, P>(band, s, g, out, nullptr);
  wave_sync();
  // strip carries (one lane per strip), as in wg_mul_mfma's closing scan
  constexpr int kStripLimbs = strip_limbs<8>();
  const uint64_t kC = (1ull << 63) - 1;
  const int w = lane;
  const bool valid = w < g.W;
  const int j0 = kStripLimbs * (valid ? w : 0);
  const uint32_t l0 = (valid && j0 < g.nout) ? out[j0] : 0u;
  const uint32_t l1 = (valid && j0 + 1 < g.nout) ? out[j0 + 1] : 0u;
  const uint64_t d = (valid && w > 0) ? (s.carry[w - 1] & kC) : 0ull;
  const bool ones = valid && (s.carry[w] >> 63);
  const uint64_t x0 = ((uint64_t)l1 << 32) | l0;
  const uint64_t x = x0 + d;
  const bool xh = x < x0;
  const bool gen = valid && xh && ones;
  const bool prop = valid && !xh && x == ~0ull && ones;
  const WaveCarry wc = wave_carry_masks(gen, prop);
  const uint32_t c = wave_carry_in(wc, 0u);
  if (valid) {
    const uint64_t y = x + c;
    const bool yh = xh || (y < x);
    if (y != x0) {
      if (j0 < g.nout) out[j0] = (uint32_t)y;
      if (j0 + 1 < g.nout) out[j0 + 1] = (uint32_t)(y >> 32);
    }
    if (yh) {
      for (int j = j0 + 2; j < min(j0 + kStripLimbs, g.nout); ++j) {
        const uint32_t v = out[j];
        out[j] = v + 1u;
        if (v != 0xffffffffu) break;
      }
    }
  }
}

}  // namespace mfma
}  // namespace bi
