/*
 * oracle.c -- plain, slow CPU reference for batched big-integer arithmetic.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load
 * or call this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * with the GPU library.
 *
 * Paper: C. E. Oancea and S. M. Watt, "High-Level Big Integer Arithmetic in
 * Futhark for GPUs".  Integers are little-endian digit arrays in base
 * B = 2^b (Section 2, Machine Model); the evaluation instantiates the digit
 * as a 64-bit unsigned word (Section 6), which is what this file computes
 * on.  The public entry points take little-endian u32 limb arrays (two u32
 * limbs are one u64 digit, an odd count is zero-padded) so that tests can
 * hand the same bytes to the GPU library and to this file.
 *
 * Every operation here has a unique mathematical result, and the oracle
 * computes that plain definition, not the GPU method:
 *   add     r = (a+b) mod 2^(32n), carry = floor((a+b)/2^(32n))
 *   sub     r = (a-b) mod 2^(32n), borrow = [a < b]
 *   mul     the full product (na+nb limbs); row-by-row schoolbook
 *   mullo   (a*b) mod 2^(32m)
 *   add6    six additions in sequence, ((((((a+b)+a)+b)+a)+b)+a) mod 2^(32n),
 *           and how many of them overflowed
 *   poly    ((a*a + b) * (b*b + b) + a*b) mod 2^(32n)
 *   divmod  q = floor(u/v), r = u - q v (Knuth, TAOCP vol. 2, 4.3.1, Alg. D)
 *   shinv   floor(B^h / v) with B = 2^32 (divmod of B^h by v)
 *   digits  the base-2^w digits of a (bit extraction)
 *   conv    c_k = sum_{i+j=k} alpha_i beta_j (double loop, 64-bit)
 *   recomb  sum_k c_k 2^(w k) as limbs (ripple accumulation)
 * Pins (tests/test_oracle_*.py) check each of these against Python's
 * arbitrary-precision integers, brute force on an edge alphabet, closed
 * forms and invariants.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ---- limb conversion: u32 pairs <-> u64 digits --------------------------- */

static int64_t n64_of(int64_t n32) { return (n32 + 1) / 2; }

static uint64_t* load64(const uint32_t* s, int64_t n32, int64_t extra)
{
    int64_t m = n64_of(n32);
    uint64_t* d = (uint64_t*)calloc((size_t)(m + extra + 1), sizeof(uint64_t));
    for (int64_t i = 0; i < n32; ++i)
        d[i / 2] |= (uint64_t)s[i] << (32 * (i % 2));
    return d;
}

static void store32(uint32_t* d, const uint64_t* s, int64_t n32)
{
    for (int64_t i = 0; i < n32; ++i)
        d[i] = (uint32_t)(s[i / 2] >> (32 * (i % 2)));
}

/* bit `pos` of a u32 limb array (0 beyond the end) */
static unsigned bit_of(const uint32_t* a, int64_t n32, int64_t pos)
{
    int64_t w = pos / 32;
    if (pos < 0 || w >= n32) return 0;
    return (a[w] >> (pos % 32)) & 1u;
}

/* ---- addition (Section 5.1: the golden map-scan-map add; here a ripple) -- */

/* r = (a + b) mod 2^(32n); *carry_out = carry out of the top limb. */
int orc_add(uint32_t* out, uint32_t* carry_out, const uint32_t* a,
            const uint32_t* b, int64_t n)
{
    int64_t m = n64_of(n);
    uint64_t *x = load64(a, n, 0), *y = load64(b, n, 0);
    uint64_t* r = (uint64_t*)calloc((size_t)m + 1, sizeof(uint64_t));
    uint64_t c = 0;
    for (int64_t i = 0; i < m; ++i) {
        u128 t = (u128)x[i] + y[i] + c;
        r[i] = (uint64_t)t;
        c = (uint64_t)(t >> 64);
    }
    /* an odd limb count leaves the top digit half used: its bit 32 is the carry */
    if (n % 2) { c = r[m - 1] >> 32; r[m - 1] &= 0xffffffffu; }
    store32(out, r, n);
    if (carry_out) *carry_out = (uint32_t)c;
    free(x); free(y); free(r);
    return 0;
}

/* ---- subtraction (Section 5.3 uses it inside `step`; mirror of add) ----- */

/* r = (a - b) mod 2^(32n); *borrow_out = [a < b]. */
int orc_sub(uint32_t* out, uint32_t* borrow_out, const uint32_t* a,
            const uint32_t* b, int64_t n)
{
    int64_t m = n64_of(n);
    uint64_t *x = load64(a, n, 0), *y = load64(b, n, 0);
    uint64_t* r = (uint64_t*)calloc((size_t)m + 1, sizeof(uint64_t));
    uint64_t br = 0;
    for (int64_t i = 0; i < m; ++i) {
        uint64_t d = x[i] - y[i];
        uint64_t b1 = x[i] < y[i];
        uint64_t d2 = d - br;
        uint64_t b2 = d < br;
        r[i] = d2;
        br = b1 | b2;
    }
    if (n % 2) { br = (r[m - 1] >> 32) ? 1u : 0u; r[m - 1] &= 0xffffffffu; }
    store32(out, r, n);
    if (borrow_out) *borrow_out = (uint32_t)br;
    free(x); free(y); free(r);
    return 0;
}

/* ---- multiplication (Section 5.2: C_k = sum_{i+j=k} A_i B_j) ------------- */

/* Full product of u64 digit arrays: r[0 .. ma+mb) = x[0..ma) * y[0..mb). */
static void mul64(uint64_t* r, const uint64_t* x, int64_t ma, const uint64_t* y,
                  int64_t mb)
{
    memset(r, 0, (size_t)(ma + mb) * sizeof(uint64_t));
    for (int64_t i = 0; i < ma; ++i) {
        uint64_t c = 0;
        for (int64_t j = 0; j < mb; ++j) {
            u128 t = (u128)x[i] * y[j] + r[i + j] + c;
            r[i + j] = (uint64_t)t;
            c = (uint64_t)(t >> 64);
        }
        r[i + mb] = c;
    }
}

/* out[0 .. na+nb) = a * b (the full product). */
int orc_mul(uint32_t* out, const uint32_t* a, int64_t na, const uint32_t* b,
            int64_t nb)
{
    int64_t ma = n64_of(na), mb = n64_of(nb);
    uint64_t *x = load64(a, na, 0), *y = load64(b, nb, 0);
    uint64_t* r = (uint64_t*)calloc((size_t)(ma + mb + 1), sizeof(uint64_t));
    mul64(r, x, ma, y, mb);
    store32(out, r, na + nb);
    free(x); free(y); free(r);
    return 0;
}

/* out[0 .. m) = (a * b) mod 2^(32m); a and b have m limbs.  The paper's
 * quadratic formula restricts i, j, k < m (Section 5.2), i.e. this product;
 * division uses it (varPrecMul / bmulG pad digits >= m with zero). */
int orc_mullo(uint32_t* out, const uint32_t* a, const uint32_t* b, int64_t m)
{
    uint32_t* full = (uint32_t*)calloc((size_t)(2 * m), sizeof(uint32_t));
    orc_mul(full, a, m, b, m);
    memcpy(out, full, (size_t)m * sizeof(uint32_t));
    free(full);
    return 0;
}

/* ---- fused workloads of the evaluation (Section 6) ----------------------- */

/* The 6-Add benchmark: six dependent additions per instance (the paper does
 * not print the expression; this one alternates the two inputs):
 * out = ((((((a+b)+a)+b)+a)+b)+a) mod 2^(32n), *overflow = the number of the
 * six additions that carried out of the top limb. */
int orc_add6(uint32_t* out, uint32_t* overflow, const uint32_t* a,
             const uint32_t* b, int64_t n)
{
    uint32_t* t = (uint32_t*)calloc((size_t)n, sizeof(uint32_t));
    uint32_t total = 0, c = 0;
    orc_add(t, &c, a, b, n);
    total += c;
    for (int step = 1; step < 6; ++step) {
        orc_add(t, &c, t, (step % 2) ? a : b, n);
        total += c;
    }
    memcpy(out, t, (size_t)n * sizeof(uint32_t));
    if (overflow) *overflow = total;
    free(t);
    return 0;
}

/* The Poly benchmark in fixed precision (products and sums mod 2^(32n), as
 * the paper's multiplication keeps the operand width):
 * out = ((a*a + b) * (b*b + b) + a*b) mod 2^(32n). */
int orc_poly(uint32_t* out, const uint32_t* a, const uint32_t* b, int64_t n)
{
    uint32_t* x = (uint32_t*)calloc((size_t)n, sizeof(uint32_t));
    uint32_t* y = (uint32_t*)calloc((size_t)n, sizeof(uint32_t));
    uint32_t* z = (uint32_t*)calloc((size_t)n, sizeof(uint32_t));
    orc_mullo(x, a, a, n);
    orc_add(x, NULL, x, b, n);          /* a*a + b */
    orc_mullo(y, b, b, n);
    orc_add(y, NULL, y, b, n);          /* b*b + b */
    orc_mullo(z, x, y, n);              /* (a*a + b)(b*b + b) */
    orc_mullo(x, a, b, n);
    orc_add(out, NULL, z, x, n);        /* + a*b */
    free(x); free(y); free(z);
    return 0;
}

/* ---- division (Section 5.3 specifies the quotient; Knuth Algorithm D) ---- */

static int64_t prec64(const uint64_t* x, int64_t m)
{
    while (m > 0 && x[m - 1] == 0) --m;
    return m;
}

static int clz64(uint64_t x)
{
    int s = 0;
    while (!(x & ((uint64_t)1 << 63))) { x <<= 1; ++s; }
    return s;
}

/* q[0..m) and r[0..n) from u[0..m), v[0..n) as u64 digits; v != 0. */
static void divmod64(uint64_t* q, uint64_t* r, const uint64_t* u, int64_t m,
                     const uint64_t* v, int64_t nv)
{
    int64_t n = prec64(v, nv), mu = prec64(u, m);
    memset(q, 0, (size_t)m * sizeof(uint64_t));
    memset(r, 0, (size_t)nv * sizeof(uint64_t));
    if (mu < n) {                         /* u < B^n <= ... : quotient 0 */
        for (int64_t i = 0; i < mu; ++i) r[i] = u[i];
        return;
    }
    if (n == 1) {                         /* short division */
        uint64_t d = v[0], rem = 0;
        for (int64_t i = mu - 1; i >= 0; --i) {
            u128 t = ((u128)rem << 64) | u[i];
            q[i] = (uint64_t)(t / d);
            rem = (uint64_t)(t % d);
        }
        r[0] = rem;
        return;
    }
    /* D1: normalise so the divisor's top digit has its high bit set */
    int s = clz64(v[n - 1]);
    uint64_t* vn = (uint64_t*)calloc((size_t)n, sizeof(uint64_t));
    uint64_t* un = (uint64_t*)calloc((size_t)mu + 1, sizeof(uint64_t));
    for (int64_t i = n - 1; i > 0; --i)
        vn[i] = (v[i] << s) | (s ? v[i - 1] >> (64 - s) : 0);
    vn[0] = v[0] << s;
    un[mu] = s ? u[mu - 1] >> (64 - s) : 0;
    for (int64_t i = mu - 1; i > 0; --i)
        un[i] = (u[i] << s) | (s ? u[i - 1] >> (64 - s) : 0);
    un[0] = u[0] << s;
    /* D2..D7: one quotient digit per position, top down */
    for (int64_t j = mu - n; j >= 0; --j) {
        u128 num = ((u128)un[j + n] << 64) | un[j + n - 1];
        u128 qhat = num / vn[n - 1];
        u128 rhat = num % vn[n - 1];
        /* D3: at most two corrections bring qhat to q or q+1 */
        while ((qhat >> 64) != 0 ||
               qhat * vn[n - 2] > ((rhat << 64) | un[j + n - 2])) {
            qhat -= 1;
            rhat += vn[n - 1];
            if ((rhat >> 64) != 0) break;
        }
        /* D4: multiply and subtract */
        uint64_t borrow = 0, carry = 0;
        for (int64_t i = 0; i < n; ++i) {
            u128 p = qhat * vn[i] + carry;
            carry = (uint64_t)(p >> 64);
            uint64_t pl = (uint64_t)p;
            uint64_t t = un[i + j] - pl;
            uint64_t b1 = un[i + j] < pl;
            uint64_t t2 = t - borrow;
            uint64_t b2 = t < borrow;
            un[i + j] = t2;
            borrow = b1 + b2;
        }
        uint64_t top = un[j + n];
        uint64_t t = top - carry;
        uint64_t b1 = top < carry;
        uint64_t t2 = t - borrow;
        uint64_t b2 = t < borrow;
        un[j + n] = t2;
        q[j] = (uint64_t)qhat;
        /* D5/D6: the rare add-back when the subtraction went negative */
        if (b1 | b2) {
            q[j] -= 1;
            uint64_t c = 0;
            for (int64_t i = 0; i < n; ++i) {
                u128 sum = (u128)un[i + j] + vn[i] + c;
                un[i + j] = (uint64_t)sum;
                c = (uint64_t)(sum >> 64);
            }
            un[j + n] += c;
        }
    }
    /* D8: unnormalise the remainder */
    for (int64_t i = 0; i < n - 1; ++i)
        r[i] = (un[i] >> s) | (s ? un[i + 1] << (64 - s) : 0);
    r[n - 1] = un[n - 1] >> s;
    free(vn); free(un);
}

/* q[0..nu) = floor(u / v), r[0..nv) = u - q v.  Returns 0, or 1 when v == 0,
 * in which case q = 0 and r = u mod 2^(32 nv). */
int orc_divmod(uint32_t* q, uint32_t* r, const uint32_t* u, int64_t nu,
               const uint32_t* v, int64_t nv)
{
    int64_t mu = n64_of(nu), mv = n64_of(nv);
    uint64_t *x = load64(u, nu, 0), *y = load64(v, nv, 0);
    if (prec64(y, mv) == 0) {
        memset(q, 0, (size_t)nu * sizeof(uint32_t));
        for (int64_t i = 0; i < nv; ++i) r[i] = i < nu ? u[i] : 0;
        free(x); free(y);
        return 1;
    }
    uint64_t* qq = (uint64_t*)calloc((size_t)mu + 1, sizeof(uint64_t));
    uint64_t* rr = (uint64_t*)calloc((size_t)mv + 1, sizeof(uint64_t));
    divmod64(qq, rr, x, mu, y, mv);
    store32(q, qq, nu);
    store32(r, rr, nv);
    free(x); free(y); free(qq); free(rr);
    return 0;
}

/* w[0 .. h+1) = floor(B^h / v) with B = 2^32: the whole shifted inverse that
 * the division of Section 5.3 computes by Newton iteration.  Returns 1 if
 * v == 0 (w = 0). */
int orc_shinv(uint32_t* w, const uint32_t* v, int64_t nv, int64_t h)
{
    uint32_t* pw = (uint32_t*)calloc((size_t)h + 1, sizeof(uint32_t));
    uint32_t* rem = (uint32_t*)calloc((size_t)nv, sizeof(uint32_t));
    pw[h] = 1;
    int st = orc_divmod(w, rem, pw, h + 1, v, nv);
    free(pw); free(rem);
    return st;
}

/* ---- the digit form of the MFMA multiply --------------------------------- */

/* out[k] = floor(a / 2^(w k)) mod 2^w for k in [0, D), read bit by bit. */
int orc_digits(uint8_t* out, const uint32_t* a, int64_t n, int w, int64_t D)
{
    for (int64_t k = 0; k < D; ++k) {
        unsigned d = 0;
        for (int t = 0; t < w; ++t)
            d |= bit_of(a, n, (int64_t)w * k + t) << t;
        out[k] = (uint8_t)d;
    }
    return 0;
}

/* c[k] = sum_{i+j=k} alpha_i beta_j for k in [0, Na+Nb-1) -- the formula of
 * Section 5.2 over small digits, with no carry handling. */
int orc_conv(int64_t* c, const uint8_t* alpha, int64_t Na, const uint8_t* beta,
             int64_t Nb)
{
    if (Na <= 0 || Nb <= 0) return 0;
    memset(c, 0, (size_t)(Na + Nb - 1) * sizeof(int64_t));
    for (int64_t i = 0; i < Na; ++i)
        for (int64_t j = 0; j < Nb; ++j)
            c[i + j] += (int64_t)alpha[i] * (int64_t)beta[j];
    return 0;
}

/* out[0..nout) = (sum_k c_k 2^(w k)) mod 2^(32 nout), c_k >= 0.  Each term is
 * added into the u32 accumulator with a ripple carry. */
int orc_recombine(uint32_t* out, int64_t nout, const int64_t* c, int64_t K, int w)
{
    memset(out, 0, (size_t)nout * sizeof(uint32_t));
    for (int64_t k = 0; k < K; ++k) {
        if (c[k] < 0) return 2;
        int64_t bit = (int64_t)w * k;
        int64_t limb = bit / 32;
        u128 v = (u128)(uint64_t)c[k] << (bit % 32);
        uint64_t carry = 0;
        for (int64_t i = limb; i < nout && (v != 0 || carry != 0); ++i) {
            uint64_t s = (uint64_t)out[i] + (uint64_t)(uint32_t)v + carry;
            out[i] = (uint32_t)s;
            carry = s >> 32;
            v >>= 32;
        }
    }
    return 0;
}
