/*
 * bigint_rocm.h -- C-ABI of a batched big-integer library for AMD MI355X
 * (gfx950).
 *
 * Method: C. E. Oancea and S. M. Watt, "High-Level Big Integer Arithmetic in
 * Futhark for GPUs".  Many independent unsigned integers of 2^15..2^19 bits
 * are processed at once, one work-group per instance (Section 2: an instance
 * fits one work-group, each work-item owning Q digits).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Limbs:      little-endian u32 limbs, instance-major: instance i of a
 *             uniform batch occupies limbs [i*n, (i+1)*n).  An array of u64
 *             digits is byte-identical to a u32 array of twice the length.
 * Ragged:     a flat limb array plus an int64 prefix-offset array `off` of
 *             length batch+1 in DEVICE memory; instance i is
 *             flat[off[i] .. off[i+1]).
 * Memory:     every data pointer is a DEVICE pointer (hipMalloc / torch CUDA
 *             tensor) unless the parameter says "host".  The caller owns all
 *             buffers; the library never frees caller memory.
 * Streams:    `stream` is a hipStream_t passed as void* (NULL = the null
 *             stream).  Calls only enqueue work on it; they do not
 *             synchronise the device, so outputs are valid once the stream
 *             has reached that point.
 * Errors:     0 = BIGINT_OK, negative = failure, and then nothing was
 *             enqueued.  Argument checks happen on the host before any
 *             launch.  Data-dependent conditions never fail a call (a zero
 *             divisor is reported per instance).  No C++ exception crosses
 *             this interface.  After BIGINT_EHIP, bigint_last_hip_error()
 *             returns the hipError_t of the failing HIP call (per thread).
 * Aliasing:   add/sub allow `out` == `a` or `out` == `b` exactly (in place);
 *             any other overlap between an output and an input, and any
 *             overlap between two outputs, is BIGINT_EINVAL.  mul and divmod
 *             outputs must not overlap any input.
 */
#ifndef BIGINT_ROCM_H
#define BIGINT_ROCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ----------------------------------------------------------- */
#define BIGINT_OK 0
#define BIGINT_EINVAL (-1)       /* bad argument: null, size <= 0, overlap, ... */
#define BIGINT_ENOMEM (-2)       /* device or host allocation failed            */
#define BIGINT_EHIP (-3)         /* a HIP runtime call failed                   */
#define BIGINT_EUNSUPPORTED (-4) /* size outside the supported range            */

/* per-instance division status (the `status` output of divmod) */
#define BIGINT_DIV_OK 0
#define BIGINT_DIVZERO 1
#define BIGINT_DIV_FAILED 2 /* an internal correction loop hit its bound; the
                               result is not valid (not expected to occur) */

/* multiplication algorithms */
#define BIGINT_MUL_AUTO 0  /* MFMA-split where supported, else plain        */
#define BIGINT_MUL_PLAIN 1 /* u64-digit schoolbook convolution               */
#define BIGINT_MUL_MFMA 2  /* 7- or 8-bit digits, int8 MFMA Toeplitz tiles   */
#define BIGINT_MUL_KARATSUBA 3 /* one Karatsuba level over BIGINT_MUL_MFMA  */

/* plan operations */
#define BIGINT_OP_MUL 1
#define BIGINT_OP_DIVMOD 2

/* plan flags */
#define BIGINT_PLAN_DEFAULT 0
#define BIGINT_PLAN_PLAIN 1   /* ragged multiply with the plain kernel        */
#define BIGINT_PLAN_NO_GRAPH 2 /* launch directly instead of a hipGraph        */

/* Largest operand (in u32 limbs) the MFMA-split multiply takes: both digit
 * arrays of an instance must fit in one work-group's 160 KiB of LDS.  With
 * 8-bit digits that holds up to 18,460 limbs; a configuration forced to
 * 7-bit digits fits up to 16,397 limbs (8 waves) or 16,831 (4 waves) and
 * beyond that returns BIGINT_EUNSUPPORTED. */
#define BIGINT_MFMA_MAX_LIMBS 18432

/* Largest dividend or divisor (in u32 limbs) the division takes: 2^19 bits.
 * Its products (up to about that many limbs per operand) run on the
 * MFMA-split multiply, whose operands must fit one work-group's LDS. */
#define BIGINT_DIV_MAX_LIMBS 16384

typedef struct bigint_plan_s* bigint_plan_t;

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int bigint_version(void);

/* Static, NUL-terminated description of a status code (never NULL). */
const char* bigint_strerror(int code);

/* The hipError_t (as int) of the last HIP failure on this thread, 0 if none. */
int bigint_last_hip_error(void);

/* ---- addition and subtraction (Section 5.1) ----------------------------------
 * The paper writes addition as map -> exclusive scan of (carry, all-ones)
 * pairs -> map (Section 5.1, golden add and baddReg); subtraction is its
 * mirror with borrows (bsubReg', used by the division step of Section 5.3).
 *
 * out[i]        = (a[i] + b[i]) mod 2^(32n)          (bigint_add)
 *               = (a[i] - b[i]) mod 2^(32n)          (bigint_sub)
 * carry_out[i]  = floor((a[i]+b[i]) / 2^(32n)) in {0,1}, or [a[i] < b[i]]
 *                 for the borrow; carry_out may be NULL.
 * a, b, out:    batch*n limbs.  carry_out: batch u32.
 * n in [1, 65536], batch >= 0 (0 enqueues nothing).  n > 65536 is
 * BIGINT_EUNSUPPORTED. */
int bigint_add(uint32_t* out, uint32_t* carry_out, const uint32_t* a,
               const uint32_t* b, int64_t n, int64_t batch, void* stream);
int bigint_sub(uint32_t* out, uint32_t* borrow_out, const uint32_t* a,
               const uint32_t* b, int64_t n, int64_t batch, void* stream);

/* ---- multiplication (Section 5.2) --------------------------------------------
 * out[i] = a[i] * b[i], the full (na+nb)-limb product.  The paper's quadratic
 * formula C_k = sum_{i+j=k} A_i B_j (Section 5.2) is evaluated either
 *   BIGINT_MUL_PLAIN: on u64 digits, each thread computing Q consecutive
 *     outputs and their balancing partners (threadConv/halfConv), partial
 *     sums kept as (low, high, carry) triples and resolved by one carry scan
 *     (bmulReg: convolution, then baddReg of the low and shifted high parts);
 *   BIGINT_MUL_MFMA: on small digits as a sum of Toeplitz-times-Hankel
 *     int8 MFMA tiles with int32 accumulation, recombined in 64-bit columns
 *     and resolved by the same carry scan.  The digit width is a tuned
 *     parameter: 7-bit digits (exact: every coefficient is at most
 *     min(Na,Nb)*127^2 < 2^31) or 8-bit digits fed as alpha - 128 (signed
 *     int8; every MFMA sum is at most min(Na,Nb)*2^14 < 2^31) with the
 *     offset terms 128 (window sums of the digits) + 2^14 (pair counts)
 *     added per coefficient in 64-bit arithmetic.  Both give the same bytes.
 *   BIGINT_MUL_KARATSUBA (na == nb >= 2): one level of Karatsuba's method
 *     over the MFMA-split multiply, with h = ceil(n/2) and s = sign(a0 - a1)
 *     sign(b1 - b0): a b = p2 B^(2h) + (p0 + p2 + s pm) B^h + p0 with
 *     p0 = a0 b0, p2 = a1 b1, pm = |a0 - a1| |b1 - b0| (three half-size
 *     products, 3/4 of the multiply-accumulates).  Not in the paper, whose
 *     conclusion names more elaborate multiplication algorithms as a next
 *     step.  The call allocates 5n limbs of workspace per instance on
 *     `stream` (stream-ordered) and frees it the same way.
 * With fewer instances than the device has CUs and no configuration forced
 * by bigint_set_mfma_config or bigint_set_mfma_tile, MFMA full products of
 * at least 32 4-strip bands (128 strips) are split: each product's bands run on
 * several work-groups (contiguous runs of about equal cost, as many as fill
 * the CUs once, at least four bands each, and only where that gives at
 * least four work-groups per instance), whose strip carry words go to a
 * workspace of 8 bytes per strip and instance allocated and freed on
 * `stream` (stream-ordered); a second launch resolves each instance's strip
 * carries.  Same bytes as one work-group per instance
 * (bigint_mfma_split_parts reports the split).
 * a: batch*na limbs, b: batch*nb limbs, out: batch*(na+nb) limbs.
 * na, nb >= 1.  MFMA needs na, nb <= BIGINT_MFMA_MAX_LIMBS (else
 * BIGINT_EUNSUPPORTED); PLAIN needs na+nb <= 32768; AUTO picks MFMA when it
 * fits and na,nb >= 64, otherwise PLAIN. */
int bigint_mul(uint32_t* out, const uint32_t* a, int64_t na, const uint32_t* b,
               int64_t nb, int64_t batch, int algo, void* stream);

/* ---- fixed-precision product and the evaluation's fused workloads (Section 6) ---
 * bigint_mullo: out[i] = a[i] * b[i] mod B^n (B = 2^32), the paper's
 *   multiplication, whose quadratic formula keeps only digits k < n
 *   (Section 5.2).  MFMA-split, computing only the strips below limb n.
 *   Small batches split each product's bands over work-groups as
 *   bigint_mul's do (same condition, workspace and bytes).
 *   a, b, out: batch*n limbs; 1 <= n <= BIGINT_MFMA_MAX_LIMBS; out must not
 *   overlap a or b.
 * bigint_add6: the 6-Add benchmark (Table tab-add): six dependent additions
 *   out[i] = ((((((a+b)+a)+b)+a)+b)+a) mod B^n = (4a + 3b) mod B^n with the
 *   operands and partial sums held in registers, so the batch moves the
 *   bytes of one addition.  overflow[i] (nullable) = how many of the six
 *   carried out of limb n-1, i.e. floor((4a + 3b) / B^n).  The paper does
 *   not print its 6-Add expression; this one alternates the two inputs.
 *   1 <= n <= 16384; out may equal a or b exactly (in place), other overlap
 *   is BIGINT_EINVAL.
 * bigint_poly: the Poly benchmark (Table tab-mul) in the paper's fixed
 *   precision: out[i] = ((a a + b)(b b + b) + a b) mod B^n, four products
 *   mod B^n and three additions per instance, one work-group per instance;
 *   the call allocates 2n limbs of workspace for each work-group of a
 *   launch (at most eight times the resident work-groups per launch) on
 *   `stream` (stream-ordered) and frees it the same way.  1 <= n <=
 *   BIGINT_MFMA_MAX_LIMBS; out must not overlap a or b. */
int bigint_mullo(uint32_t* out, const uint32_t* a, const uint32_t* b, int64_t n,
                 int64_t batch, void* stream);
int bigint_add6(uint32_t* out, uint32_t* overflow, const uint32_t* a,
                const uint32_t* b, int64_t n, int64_t batch, void* stream);
int bigint_poly(uint32_t* out, const uint32_t* a, const uint32_t* b, int64_t n,
                int64_t batch, void* stream);

/* ---- division (Section 5.3) ------------------------------------------------------
 * q[i] = floor(u[i] / v[i]), r[i] = u[i] - q[i]*v[i], 0 <= r[i] < v[i].
 * The quotient comes from the whole shifted inverse w ~ B^h / v (B = 2^32,
 * h = precision of u), grown by the paper's signed Newton `step` (Section
 * 5.3, both branches, one guard limb, no exact fix-up on the way) whose
 * multiplications run on the MFMA-split multiply; then q~ = floor(u*w / B^h)
 * and the signed remainder u - q~ v brought into [0, v) by a few unit
 * corrections.
 * u: batch*nu limbs, v: batch*nv limbs, q: batch*nu limbs, r: batch*nv limbs,
 * status: batch int32 or NULL.  A zero divisor gives status BIGINT_DIVZERO,
 * q = 0 and r = u mod 2^(32 nv); the call itself still returns BIGINT_OK.
 * nu, nv in [1, BIGINT_DIV_MAX_LIMBS] (else BIGINT_EUNSUPPORTED).  The call allocates its
 * workspace with hipMallocAsync on `stream`. */
int bigint_divmod(uint32_t* q, uint32_t* r, int32_t* status, const uint32_t* u,
                  int64_t nu, const uint32_t* v, int64_t nv, int64_t batch,
                  void* stream);

/* bigint_divmod_noalloc: bigint_divmod (same arguments, same results, same
 * size limits) for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * It calls no allocation routine.  Its workspace is a fixed array of
 * 128 MiB in device memory that each GPU the library runs on holds until the
 * process ends; a batch whose divisions need more workspace slots than that
 * array holds at once runs in several consecutive launches on `stream`.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (different streams or threads) race and must not be issued.
 * The first call on a device looks up the array's address there
 * (hipGetSymbolAddress); a failure is BIGINT_EHIP. */
int bigint_divmod_noalloc(uint32_t* q, uint32_t* r, int32_t* status,
                          const uint32_t* u, int64_t nu, const uint32_t* v,
                          int64_t nv, int64_t batch, void* stream);

/* ---- plans for ragged batches ------------------------------------------------------
 * A plan fixes the instance sizes of a ragged batch (host arrays len_a, len_b
 * of `batch` limb counts; for DIVMOD len_a are the dividend and len_b the
 * divisor lengths), bins instances by cost, orders them largest first (a
 * division plan reverses every other row of the work-groups resident at the
 * start, so that the largest divisions share their CUs with the smallest) and
 * picks a tuned tile configuration per bin (from the autotune cache if one
 * was loaded, else built-in defaults).  Creating a plan allocates a small
 * device schedule; the plan owns it until bigint_plan_destroy.
 * Workspace: bigint_plan_workspace_size reports the device scratch a call
 * needs (a multiply plan needs some only when a segment is split: 8 bytes per
 * strip of its instances); pass a buffer of at least that size with
 * bigint_plan_set_workspace, otherwise the first call allocates one (owned
 * by the plan).
 * A plan must not be used by two streams at once. */
int bigint_plan_create(bigint_plan_t* plan, int op, const int64_t* len_a,
                       const int64_t* len_b, int64_t batch, int flags);
int bigint_plan_workspace_size(bigint_plan_t plan, size_t* bytes);
int bigint_plan_set_workspace(bigint_plan_t plan, void* dev, size_t bytes);
int bigint_plan_destroy(bigint_plan_t plan);

/* Diagnostic counters of a plan, written to info[0 .. n) (host int64; n <= 3
 * are defined, further entries are set to 0): [0] kernel launches one call
 * enqueues, [1] hipGraphs instantiated so far (one per new set of call
 * pointers), [2] calls so far that launched an already instantiated graph.
 * Lets a caller confirm that repeated calls replay a captured graph. */
int bigint_plan_info(bigint_plan_t plan, int64_t* info, int n);

/* Ragged multiplication: out instance i = a instance i * b instance i, with
 * out_off[i+1]-out_off[i] == (a_off[i+1]-a_off[i]) + (b_off[i+1]-b_off[i]);
 * the limb counts must equal those given to bigint_plan_create (not checked
 * on the device).  The instances run largest first, one work-group each, in
 * a few launches (one per run of instances sharing a tile configuration,
 * each also taking some smaller instances to fill its end); the launches are
 * captured into a hipGraph and replayed on later calls with the same
 * pointers (unless BIGINT_PLAN_NO_GRAPH).  Offsets are DEVICE int64 arrays
 * of length batch+1. */
int bigint_mul_ragged(uint32_t* out, const int64_t* out_off, const uint32_t* a,
                      const int64_t* a_off, const uint32_t* b,
                      const int64_t* b_off, int64_t batch, bigint_plan_t plan,
                      void* stream);

/* The segments of a ragged multiply plan (diagnostic): *n_segments = the
 * launches one bigint_mul_ragged call makes on the MFMA-split path (0 for a
 * plain or division plan), and for segment k < max_segments the host int64
 * row seg[9k .. 9k+9): [0] first queue position (queue = instances largest
 * first), [1] instances, [2] digit bits, [3] strips per band of its leading
 * configuration, [4] waves per work-group, [5] work-groups resident at once,
 * [6] digit products its instances compute (sum of Na*Nb at its digit width),
 * [7] modelled busy fraction in parts per million: the segment's cost (sum
 * of la*lb) over resident work-groups times the span of the plan's largest-
 * first list schedule, [8] work-groups per instance: 1, or the parts of a
 * segment of few instances whose bands are split as bigint_mul splits a
 * small batch (then 4 strips per band and 4 waves, and two launches).  The
 * plan's load-balance figure per launch. */
int bigint_plan_segments(bigint_plan_t plan, int64_t* seg, int max_segments,
                         int* n_segments);

/* One segment of a ragged multiply (same arguments as bigint_mul_ragged,
 * segment < the count bigint_plan_segments reports): launches only that
 * segment's kernel, directly (no graph), writing only the products of its
 * instances.  Running every segment once, in any order, equals one
 * bigint_mul_ragged call; lets a caller time or overlap segments. */
int bigint_mul_ragged_segment(uint32_t* out, const int64_t* out_off,
                              const uint32_t* a, const int64_t* a_off,
                              const uint32_t* b, const int64_t* b_off,
                              int64_t batch, bigint_plan_t plan, int segment,
                              void* stream);

/* Ragged division: instance i divides u[u_off[i]..) by v[v_off[i]..); q
 * instance i has the dividend's limb count and r the divisor's.  The
 * division launches (one or more, each at most eight times the work-groups
 * that stay resident, one workspace slot each) are captured into a hipGraph
 * and replayed like the ragged multiply's (unless BIGINT_PLAN_NO_GRAPH). */
int bigint_divmod_ragged(uint32_t* q, const int64_t* q_off, uint32_t* r,
                         const int64_t* r_off, int32_t* status,
                         const uint32_t* u, const int64_t* u_off,
                         const uint32_t* v, const int64_t* v_off, int64_t batch,
                         bigint_plan_t plan, void* stream);

/* ---- autotuning ----------------------------------------------------------------
 * Times every candidate tile configuration of the MFMA-split multiply on the
 * current device for each size bin (2^12..2^19 bits): strips per band,
 * waves per work-group, digit width and MFMA tile (16x16x64 or 32x32x32,
 * the "chunk width"); keeps the fastest and
 * writes the table as JSON to `cache_path` (host path; NULL = do not write).
 * Later plans use the table.  bigint_autotune_load reads such a file (a
 * NULL path restores the built-in table).  All candidates produce identical
 * bytes; the table only affects speed.
 * Environment: BIGINT_TUNE_CACHE=<path> loads such a table once, before the
 * library's first table lookup (a later bigint_autotune or
 * bigint_autotune_load replaces it); a file that does not parse leaves the
 * built-in table (bigint_autotune_load on the same path reports why).
 * BIGINT_DEBUG=1 prints one line on stderr per configuration the library
 * picks: each MFMA-split, plain or Karatsuba multiply call (digit width,
 * tile, strips per band, waves, work-groups per product), each segment of a
 * ragged multiply plan and each division plan. */
int bigint_autotune(const char* cache_path, int flags);
int bigint_autotune_load(const char* cache_path);

/* ---- diagnostics: the steps of the MFMA-split multiply ---------------------------
 * bigint_digits7: out[i*D + k] = floor(a[i] / 2^(7k)) mod 128 for k < D
 *   (the digit split); a: batch*n limbs, out: batch*D bytes, D >= 1.
 * bigint_conv7: c[i*(Na+Nb-1) + k] = sum_{s+t=k} alpha_s beta_t over the
 *   7-bit digits of a[i] (Na = ceil(32na/7)) and b[i] (Nb = ceil(32nb/7)),
 *   computed by the int8 MFMA tiles (int32 output, before recombination).
 * bigint_shinv: w[i*(h+1) ..] = floor(B^h / v[i]) with B = 2^32, the whole
 *   shifted inverse of the division; v: batch*nv limbs, needs h >= nv and
 *   a nonzero top limb of v (else that instance's w is 0);
 *   h <= BIGINT_DIV_MAX_LIMBS. */
int bigint_digits7(uint8_t* out, const uint32_t* a, int64_t n, int64_t D,
                   int64_t batch, void* stream);
int bigint_conv7(int32_t* c, const uint32_t* a, int64_t na, const uint32_t* b,
                 int64_t nb, int64_t batch, void* stream);
int bigint_shinv(uint32_t* w, const uint32_t* v, int64_t nv, int64_t h,
                 int64_t batch, void* stream);

/* bigint_diag_divmod_ragged: bigint_divmod_ragged (same arguments, same
 * results) that also writes, per division, four counters of the procedure
 * of Section 5.3 to counts[4*i .. 4*i+3] (device int64, 4*batch, must not
 * overlap q or r): [0] the Newton steps (`step`) taken, [1] those taken on
 * the negative branch (e = B^c - V w <= 0: w B^m minus a ceiling), [2] the
 * unit corrections of the quotient (adding or subtracting v from the signed
 * remainder; bounded loops, and hitting a bound marks the division
 * BIGINT_DIV_FAILED), [3] the int8 multiply-accumulates of the
 * division's MFMA products: for each product, the digit pairs (i, j) whose
 * coefficient i + j lies in the strips it computes (products of operands of
 * at most 64 limbs run on the vector ALU and add none).  Divisions that need
 * no Newton iteration (v < B, u < v, v = 0) report zeros.  Launches
 * directly (no graph). */
int bigint_diag_divmod_ragged(int64_t* counts, uint32_t* q, const int64_t* q_off,
                              uint32_t* r, const int64_t* r_off, int32_t* status,
                              const uint32_t* u, const int64_t* u_off,
                              const uint32_t* v, const int64_t* v_off,
                              int64_t batch, bigint_plan_t plan, void* stream);

/* Register-only int8 MFMA rate probe: `blocks` work-groups of 4 waves, each
 * wave issuing 64 v_mfma_i32_16x16x64_i8 per iteration (8 independent
 * accumulators, 16384 multiply-accumulates each) for `iters` iterations, no
 * memory traffic.  toggle bit 0 flips the operand bit patterns between
 * rounds of 8 (random data draws more power than constant data); toggle
 * bit 1 runs v_mfma_i32_32x32x32_i8 instead (4 accumulators per wave, 32
 * MFMAs of 32,768 multiply-accumulates per iteration: the same work per
 * iteration).
 * scratch: blocks*256 int32 (results kept so the work is not removed).
 * Time it with events on `stream` to get the achievable MFMA rate. */
int bigint_diag_mfma_rate(int32_t* scratch, int64_t blocks, int64_t iters, int toggle,
                          void* stream);

/* Register-only rate probe of the plain multiply's inner operation, the
 * 32x32-bit product added to a 64-bit value (v_mad_u64_u32): `blocks`
 * work-groups of 4 waves, each lane running 8 independent chains of 64 such
 * operations per iteration for `iters` iterations, no memory traffic.
 * scratch: blocks*256 uint64 (results kept so the work is not removed).
 * Time it with events on `stream`: blocks*256*iters*64 operations. */
int bigint_diag_mad_rate(uint64_t* scratch, int64_t blocks, int64_t iters, void* stream);

/* Tile parameters of the MFMA multiply used by the next calls on this thread
 * (strips per wave band: 4, 8 or 16, or 32 with 32x32 tiles; waves per
 * work-group: 4 or 8, or 1 for
 * one wave per instance with four instances per work-group -- the paper's
 * ipb instances per block -- which bigint_mul and bigint_mullo use with
 * 8-bit digits when na + nb <= 4096 limbs and otherwise treat as 4; digit
 * width: 7 or 8 bits); 0 keeps the tuned default.  Plans read the tuned
 * table only.  Exists so tests can check that every configuration gives the
 * same bytes; other values return BIGINT_EINVAL. */
int bigint_set_mfma_config(int strips_per_band, int waves, int digit_bits);

/* MFMA tile of the next calls on this thread: 16 (v_mfma_i32_16x16x64_i8,
 * the default) or 32 (v_mfma_i32_32x32x32_i8: a 32x32 result tile of 1024
 * digit coefficients, four strips, with twice the multiply-accumulates per
 * instruction for the same operand bytes); 0 keeps the tuned choice.  The
 * 32x32 tile serves bigint_mul and bigint_mullo with 8-bit digits and 8 or
 * 16 strips per band on a work-group per instance, where its LDS fits (its
 * zero padding is wider: 18,432-limb operands on 8 waves do not); every other
 * configuration (and the ragged, Karatsuba, Poly and division kernels) runs
 * 16x16 tiles.  Both tiles give the same bytes.  Other values return
 * BIGINT_EINVAL.  bigint_mfma_tile returns the tile bigint_mul would use for
 * an na x nb product on this thread (16 or 32), or a negative status. */
int bigint_set_mfma_tile(int tile);
int bigint_mfma_tile(int64_t na, int64_t nb);

/* The tile configuration bigint_mul would use on this thread for an na x nb
 * product (tuned table, then this thread's overrides), written to the three
 * host ints.  Where the table gives one wave per instance, bigint_mul runs
 * it only for batches of at least na*nb/64 instances, bigint_mullo for at
 * least n*n/256, bigint_poly for at least n*n/16, and 4 waves per instance
 * below that (one
 * wave per instance leaves most CUs idle on small batches).  bigint_mul and
 * bigint_mullo on a batch of fewer instances than the device has CUs run 8
 * waves where this reports 4 (and 4 strips per band where it reports one
 * wave, and always for bigint_mullo), if the LDS allows.  A wave count set with bigint_set_mfma_config is used at every
 * batch.  BIGINT_EUNSUPPORTED if the MFMA multiply does not take that
 * size with it; BIGINT_EINVAL for null pointers or sizes < 1. */
/* Work-groups per instance that bigint_mul's MFMA path gives a batch of
 * `batch` full na x nb products on the current device (1: one work-group
 * per instance; more: the bands split as described at bigint_mul), written
 * to the host int.  BIGINT_EINVAL for null pointers or sizes < 1. */
int bigint_mfma_split_parts(int64_t na, int64_t nb, int64_t batch, int* parts);

int bigint_mfma_config(int64_t na, int64_t nb, int* strips_per_band, int* waves,
                       int* digit_bits);

#ifdef __cplusplus
}
#endif
#endif /* BIGINT_ROCM_H */
