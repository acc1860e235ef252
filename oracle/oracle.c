/*
 * oracle.c -- plain, slow, bit-by-bit CPU reference of the block-wise
 * inner-product extractor.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or
 * constant generator with the HIP library.
 *
 * What it computes (Li & Zhou, "Real-Time Seedless Post-Processing for
 * Quantum Random Number Generators"):
 *
 *   * Sec. 3.2, Def. 3.2 (inner-product extractor): for x, y in (F_{2^q})^n,
 *     Ext_IP(x, y) = sum_i x_i * y_i, with field addition = bitwise parity
 *     (Sec. 3.2, the identification of F_{2^q} with {0,1}^q) and field
 *     multiplication in F_{2^q}.
 *   * Algorithm 1 (equal blocks): the raw data of each source is cut into
 *     consecutive blocks of q*n bits; block l of X is paired with block l of
 *     Y and each pair yields the q-bit output Z^(l); the outputs are
 *     concatenated in block order (Thm. 3.6 / Thm. 3.7 output Z^(1) o Z^(2) ...).
 *
 * Readings where the paper is silent (all fixed here, one place each):
 *   - field basis: polynomial basis, bit j of an element <-> coefficient of t^j,
 *     F_{2^q} = GF(2)[t] / (P) for a fixed irreducible P of degree q;
 *   - bit order: bit r of a block is bit (r mod 8) of byte r/8 (LSB first);
 *   - element i of a block occupies block bits [i*q, (i+1)*q);
 *   - block l occupies stream bits [l*qn, (l+1)*qn) -- consecutive,
 *     non-overlapping blocks (the index update of Algorithm 1 read as
 *     advancing by one whole block, as Algorithm 2 does);
 *   - output coefficient j of Z^(l) is output stream bit l*q + j;
 *   - a trailing partial block is not processed.
 *
 * Every product below is computed one bit at a time (one bit per byte), with
 * no word-level tricks, so that the code can be checked against the
 * definition by eye.  The polynomial helpers at the end (irreducibility test
 * and modulus search) use 64-bit words for speed; they only fix the modulus
 * convention and are pinned separately by the tests.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* ------------------------------------------------------------------------ */
/* bit access, LSB first                                                    */
/* ------------------------------------------------------------------------ */
static int get_bit(const uint8_t *buf, uint64_t r)
{
    return (buf[r >> 3] >> (r & 7)) & 1;
}

static void put_bit(uint8_t *buf, uint64_t r, int v)
{
    uint8_t m = (uint8_t)(1u << (r & 7));
    if (v)
        buf[r >> 3] |= m;
    else
        buf[r >> 3] &= (uint8_t)~m;
}

/* exps: every exponent of P, including q and 0, distinct, in any order. */
static int check_modulus(uint32_t q, const uint32_t *exps, uint32_t n_exps)
{
    int has_q = 0, has_0 = 0;
    if (q == 0 || exps == NULL || n_exps < 2)
        return 0;
    for (uint32_t i = 0; i < n_exps; i++) {
        if (exps[i] > q)
            return 0;
        if (exps[i] == q)
            has_q = 1;
        if (exps[i] == 0)
            has_0 = 1;
        for (uint32_t j = 0; j < i; j++)
            if (exps[j] == exps[i])
                return 0;
    }
    return has_q && has_0;
}

/*
 * One block pair, bit by bit.
 *   xb, yb : n_e*q bits each, one bit per byte (element i = bits [iq, iq+q))
 *   c      : scratch of 2q-1 bytes
 *   z      : q bytes out, one bit per byte
 */
static void ext_ip_bits(const uint8_t *xb, const uint8_t *yb, uint32_t n_e,
                        uint32_t q, const uint32_t *exps, uint32_t n_exps,
                        uint8_t *c, uint8_t *z)
{
    memset(c, 0, 2 * (size_t)q - 1);
    /* Unreduced sum of products: field addition is XOR and reduction mod P
     * is linear, so sum_i (x_i * y_i mod P) = (sum_i x_i * y_i) mod P.
     * c[k] = XOR_i XOR_{j+l=k} x_i[j] AND y_i[l]. */
    for (uint32_t i = 0; i < n_e; i++) {
        const uint8_t *xi = xb + (size_t)i * q;
        const uint8_t *yi = yb + (size_t)i * q;
        for (uint32_t j = 0; j < q; j++)
            for (uint32_t l = 0; l < q; l++)
                c[j + l] ^= (uint8_t)(xi[j] & yi[l]);
    }
    /* Reduce mod P: clear the top coefficients one at a time, each time
     * adding t^(d-q) * P. */
    for (int64_t d = 2 * (int64_t)q - 2; d >= (int64_t)q; d--) {
        if (c[d])
            for (uint32_t e = 0; e < n_exps; e++)
                c[d - q + exps[e]] ^= 1;
    }
    for (uint32_t j = 0; j < q; j++)
        z[j] = c[j];
}

/*
 * Algorithm 1 over a whole stream pair.
 *   x, y      : raw bytes of the two sources
 *   n_pairs   : number of block pairs to process (the caller passes
 *               floor(8*len/n_bits))
 *   n_bits    : block length n in bits (= n_e * q)
 *   q         : field degree = output bits per block
 *   exps      : exponents of P (see check_modulus)
 *   out       : ceil(n_pairs*q/8) bytes; bits are written one by one
 */
int orc_ext_blocks(const uint8_t *x, const uint8_t *y, uint64_t n_pairs,
                   uint64_t n_bits, uint32_t q, const uint32_t *exps,
                   uint32_t n_exps, uint8_t *out)
{
    if (!check_modulus(q, exps, n_exps) || n_bits == 0 || n_bits % q)
        return ORC_EINVAL;
    if (n_pairs == 0)
        return ORC_OK;
    if (!x || !y || !out)
        return ORC_EINVAL;
    uint32_t n_e = (uint32_t)(n_bits / q);
    uint8_t *xb = malloc(n_bits), *yb = malloc(n_bits);
    uint8_t *c = malloc(2 * (size_t)q), *z = malloc(q);
    if (!xb || !yb || !c || !z) {
        free(xb); free(yb); free(c); free(z);
        return ORC_ENOMEM;
    }
    for (uint64_t l = 0; l < n_pairs; l++) {
        for (uint64_t r = 0; r < n_bits; r++) {
            xb[r] = (uint8_t)get_bit(x, l * n_bits + r);
            yb[r] = (uint8_t)get_bit(y, l * n_bits + r);
        }
        ext_ip_bits(xb, yb, n_e, q, exps, n_exps, c, z);
        for (uint32_t j = 0; j < q; j++)
            put_bit(out, l * (uint64_t)q + j, z[j]);
    }
    free(xb); free(yb); free(c); free(z);
    return ORC_OK;
}

/*
 * Same as orc_ext_blocks but only for the block pairs listed in idx[]
 * (outputs written densely, q bits per listed pair, pair k at bits [kq,(k+1)q)).
 * Used to check sampled blocks of large workloads.
 */
int orc_ext_sampled(const uint8_t *x, const uint8_t *y, const uint64_t *idx,
                    uint64_t n_idx, uint64_t n_bits, uint32_t q,
                    const uint32_t *exps, uint32_t n_exps, uint8_t *out)
{
    if (!check_modulus(q, exps, n_exps) || n_bits == 0 || n_bits % q)
        return ORC_EINVAL;
    if (n_idx == 0)
        return ORC_OK;
    uint32_t n_e = (uint32_t)(n_bits / q);
    uint8_t *xb = malloc(n_bits), *yb = malloc(n_bits);
    uint8_t *c = malloc(2 * (size_t)q), *z = malloc(q);
    if (!xb || !yb || !c || !z) {
        free(xb); free(yb); free(c); free(z);
        return ORC_ENOMEM;
    }
    for (uint64_t k = 0; k < n_idx; k++) {
        uint64_t l = idx[k];
        for (uint64_t r = 0; r < n_bits; r++) {
            xb[r] = (uint8_t)get_bit(x, l * n_bits + r);
            yb[r] = (uint8_t)get_bit(y, l * n_bits + r);
        }
        ext_ip_bits(xb, yb, n_e, q, exps, n_exps, c, z);
        for (uint32_t j = 0; j < q; j++)
            put_bit(out, k * (uint64_t)q + j, z[j]);
    }
    free(xb); free(yb); free(c); free(z);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Modulus convention: irreducibility test and the lowest-weight search.    */
/* Word-level GF(2)[t] arithmetic, 64 coefficients per word, LSB = t^0.     */
/* ------------------------------------------------------------------------ */

static int poly_deg(const uint64_t *a, int nw)
{
    for (int i = nw - 1; i >= 0; i--)
        if (a[i])
            return i * 64 + 63 - __builtin_clzll(a[i]);
    return -1;
}

/* dst ^= src << s (multi-word), dst has dw words, src has sw words */
static void xor_shifted(uint64_t *dst, int dw, const uint64_t *src, int sw,
                        uint32_t s)
{
    int ws = (int)(s >> 6), bs = (int)(s & 63);
    for (int i = 0; i < sw; i++) {
        uint64_t v = src[i];
        if (!v)
            continue;
        int p = i + ws;
        if (p < dw)
            dst[p] ^= v << bs;
        if (bs && p + 1 < dw)
            dst[p + 1] ^= v >> (64 - bs);
    }
}

/* Reduce t (tw words, any degree < 64*tw) modulo P = sum t^exps[i] of degree
 * q, using t^q = sum_{e != q} t^e repeatedly on the part of degree >= q.
 * hi is scratch of tw words.  Requires every non-leading exponent < q. */
static void reduce_sparse(uint64_t *t, int tw, uint32_t q, const uint32_t *exps,
                          uint32_t n_exps, uint64_t *hi)
{
    for (;;) {
        int d = poly_deg(t, tw);
        if (d < (int)q)
            return;
        /* hi = t >> q ; then clear bits >= q of t */
        memset(hi, 0, sizeof(uint64_t) * tw);
        int ws = (int)(q >> 6), bs = (int)(q & 63);
        for (int i = ws; i < tw; i++) {
            uint64_t v = t[i] >> bs;
            if (bs && i + 1 < tw)
                v |= t[i + 1] << (64 - bs);
            hi[i - ws] = v;
        }
        if (bs) {
            t[ws] &= (1ull << bs) - 1;
            ws++;
        }
        for (int i = ws; i < tw; i++)
            t[i] = 0;
        for (uint32_t k = 0; k < n_exps; k++)
            if (exps[k] != q)
                xor_shifted(t, tw, hi, tw, exps[k]);
    }
}

/* r = a^2 mod P, P given by exponent list (P = sum t^exps[i], deg q).
 * a has degree < q.  r and a may alias.  tmp has room for 2q+64 bits,
 * hi likewise. */
static void sqr_mod(uint64_t *r, const uint64_t *a, uint32_t q,
                    const uint32_t *exps, uint32_t n_exps, uint64_t *tmp,
                    uint64_t *hi)
{
    static uint16_t spread[256];
    static int ready = 0;
    if (!ready) {
        /* squaring in characteristic 2 moves coefficient i to 2i */
        for (int v = 0; v < 256; v++) {
            uint16_t s = 0;
            for (int b = 0; b < 8; b++)
                if ((v >> b) & 1)
                    s |= (uint16_t)(1u << (2 * b));
            spread[v] = s;
        }
        ready = 1;
    }
    int nw = (int)((q + 63) / 64);
    int tw = 2 * nw + 1;
    memset(tmp, 0, sizeof(uint64_t) * tw);
    for (int i = 0; i < nw; i++) {
        uint64_t w = a[i], lo = 0, hi2 = 0;
        for (int b = 0; b < 4; b++) {
            lo |= (uint64_t)spread[(w >> (8 * b)) & 255] << (16 * b);
            hi2 |= (uint64_t)spread[(w >> (8 * b + 32)) & 255] << (16 * b);
        }
        tmp[2 * i] = lo;
        tmp[2 * i + 1] = hi2;
    }
    reduce_sparse(tmp, tw, q, exps, n_exps, hi);
    memcpy(r, tmp, sizeof(uint64_t) * nw);
}

/* a = a mod b in place (b nonzero); both have nw words. */
static void poly_mod(uint64_t *a, const uint64_t *b, int nw)
{
    int db = poly_deg(b, nw);
    for (;;) {
        int da = poly_deg(a, nw);
        if (da < db)
            return;
        xor_shifted(a, nw, b, nw, (uint32_t)(da - db));
    }
}

/* 1 if gcd(a, b) == 1 (a, b destroyed), nw words each. */
static int coprime(uint64_t *a, uint64_t *b, int nw)
{
    for (;;) {
        if (poly_deg(b, nw) < 0)
            return poly_deg(a, nw) == 0;
        poly_mod(a, b, nw);
        uint64_t *t = a;
        a = b;
        b = t;
    }
}

/*
 * Rabin's irreducibility test: P of degree q is irreducible over GF(2) iff
 * t^(2^q) = t (mod P) and gcd(t^(2^(q/r)) - t, P) = 1 for every prime r | q.
 * Returns 1 irreducible, 0 reducible, <0 error.
 */
int orc_is_irreducible(uint32_t q, const uint32_t *exps, uint32_t n_exps)
{
    if (!check_modulus(q, exps, n_exps))
        return ORC_EINVAL;
    if (q == 1)
        return 1;
    int nw = (int)((q + 64) / 64) + 1; /* room for P itself (degree q) */
    uint64_t *h = calloc(nw, 8), *tmp = calloc(2 * nw + 2, 8);
    uint64_t *hi = calloc(2 * nw + 2, 8);
    uint64_t *g1 = calloc(nw, 8), *g2 = calloc(nw, 8);
    uint32_t primes[32];
    int np = 0;
    if (!h || !tmp || !hi || !g1 || !g2) {
        free(h); free(tmp); free(hi); free(g1); free(g2);
        return ORC_ENOMEM;
    }
    uint32_t m = q;
    for (uint32_t r = 2; r * r <= m; r++)
        if (m % r == 0) {
            primes[np++] = r;
            while (m % r == 0)
                m /= r;
        }
    if (m > 1)
        primes[np++] = m;

    int result = 1;
    /* For each prime r | q: h = t^(2^(q/r)) mod P, then gcd(h - t, P). */
    for (int k = 0; k < np && result; k++) {
        memset(h, 0, nw * 8);
        h[0] = 2; /* t (q >= 2) */
        for (uint32_t s = 0; s < q / primes[k]; s++)
            sqr_mod(h, h, q, exps, n_exps, tmp, hi);
        memcpy(g1, h, nw * 8);
        g1[0] ^= 2; /* h - t */
        memset(g2, 0, nw * 8);
        for (uint32_t e = 0; e < n_exps; e++)
            g2[exps[e] >> 6] ^= 1ull << (exps[e] & 63);
        if (poly_deg(g1, nw) < 0 || !coprime(g1, g2, nw))
            result = 0;
    }
    if (result) {
        memset(h, 0, nw * 8);
        h[0] = 2;
        for (uint32_t s = 0; s < q; s++)
            sqr_mod(h, h, q, exps, n_exps, tmp, hi);
        h[0] ^= 2;
        if (poly_deg(h, nw) >= 0)
            result = 0;
    }
    free(h); free(tmp); free(hi); free(g1); free(g2);
    return result;
}

/* Small-degree helpers for the sieve: polynomials of degree <= 16 in a
 * uint32 (bit i = coefficient of t^i). */
static uint32_t small_mulmod(uint32_t a, uint32_t b, uint32_t f, int df)
{
    uint32_t r = 0;
    while (b) {
        if (b & 1)
            r ^= a;
        b >>= 1;
        a <<= 1;
        if ((a >> df) & 1)
            a ^= f;
    }
    return r;
}

static uint32_t small_pow_t(uint32_t e, uint32_t f, int df)
{
    /* t^e mod f by square and multiply */
    uint32_t r = 1, base = 2;
    if (df == 1)
        base = 2 ^ f; /* t mod (t + c) */
    while (e) {
        if (e & 1)
            r = small_mulmod(r, base, f, df);
        base = small_mulmod(base, base, f, df);
        e >>= 1;
    }
    return r;
}

static int small_deg(uint32_t a)
{
    return a ? 31 - __builtin_clz(a) : -1;
}

static uint32_t small_mod(uint32_t a, uint32_t f)
{
    int df = small_deg(f);
    while (small_deg(a) >= df)
        a ^= f << (small_deg(a) - df);
    return a;
}

/* list every irreducible polynomial of degree 1..maxdeg by trial division */
static int list_irreducibles(int maxdeg, uint32_t *out, int cap)
{
    int n = 0;
    for (uint32_t f = 2; f < (1u << (maxdeg + 1)); f++) {
        int df = small_deg(f), irr = 1;
        for (int k = 0; k < n && irr; k++) {
            if (2 * small_deg(out[k]) > df)
                break;
            if (small_mod(f, out[k]) == 0)
                irr = 0;
        }
        if (irr) {
            if (n >= cap)
                return n;
            out[n++] = f;
        }
    }
    return n;
}

/*
 * Modulus convention: the lowest-weight irreducible P of degree q, and
 * among those of that weight the lexicographically smallest exponent tuple
 * (a trinomial t^q + t^a + 1 with least a if any exists, else a pentanomial
 * t^q + t^a + t^b + t^c + 1, q > a > b > c > 0, least a, then b, then c).
 * Writes the exponents in decreasing order (q first, 0 last) to out_exps
 * (room for 5) and returns their count, or <= 0 if none was found
 * (degrees below 2 have no such modulus in this convention).
 */
int orc_find_modulus(uint32_t q, uint32_t *out_exps)
{
    enum { SIEVE_DEG = 14, CAP = 2048 };
    static uint32_t irr[CAP];
    static int n_irr = 0;
    if (q < 2 || !out_exps)
        return ORC_EINVAL;
    if (!n_irr)
        n_irr = list_irreducibles(SIEVE_DEG, irr, CAP);
    /* tq[k] = t^q mod irr[k]; pw[k][e] computed on demand */
    uint32_t *tq = malloc(sizeof(uint32_t) * n_irr);
    if (!tq)
        return ORC_ENOMEM;
    for (int k = 0; k < n_irr; k++)
        tq[k] = small_pow_t(q, irr[k], small_deg(irr[k]));

    /* trinomials.  The reciprocal t^q P(1/t) of an irreducible P with
     * nonzero constant term is irreducible, and maps t^q + t^a + 1 to
     * t^q + t^(q-a) + 1, so the least a of an irreducible trinomial is at
     * most q/2: no need to look further. */
    for (uint32_t a = 1; 2 * a <= q; a++) {
        uint32_t e[3] = {q, a, 0};
        int sieved = 0;
        for (int k = 0; k < n_irr && !sieved; k++) {
            int df = small_deg(irr[k]);
            if ((uint32_t)df >= q)
                break;
            uint32_t v = tq[k] ^ small_pow_t(a, irr[k], df) ^ 1;
            if (v == 0)
                sieved = 1;
        }
        if (sieved)
            continue;
        if (orc_is_irreducible(q, e, 3) == 1) {
            memcpy(out_exps, e, sizeof e);
            free(tq);
            return 3;
        }
    }
    /* pentanomials */
    for (uint32_t a = 3; a < q; a++)
        for (uint32_t b = 2; b < a; b++)
            for (uint32_t c = 1; c < b; c++) {
                uint32_t e[5] = {q, a, b, c, 0};
                int sieved = 0;
                for (int k = 0; k < n_irr && !sieved; k++) {
                    int df = small_deg(irr[k]);
                    if ((uint32_t)df >= q)
                        break;
                    uint32_t v = tq[k] ^ small_pow_t(a, irr[k], df) ^
                                 small_pow_t(b, irr[k], df) ^
                                 small_pow_t(c, irr[k], df) ^ 1;
                    if (v == 0)
                        sieved = 1;
                }
                if (sieved)
                    continue;
                if (orc_is_irreducible(q, e, 5) == 1) {
                    memcpy(out_exps, e, sizeof e);
                    free(tq);
                    return 5;
                }
            }
    free(tq);
    return 0;
}
