/*
 * Plain CPU oracle for the RNS-CKKS arithmetic under the column-wise
 * encrypted-inference path (Volley Revolver, Inference++).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or generator with
 * the HIP library.
 *
 * Style: every routine is the textbook definition, written with unsigned
 * __int128 products and the '%' operator, single threaded, no blocking and no
 * lazy reduction.  Polynomials live in the coefficient domain; the NTT here is
 * only a tool for negacyclic products (and is pinned against the direct
 * evaluation definition and the schoolbook product in the tests).
 *
 * The HE operations come from the paper's preliminaries (Enc, Dec, Add, Mul,
 * cMul, Rot, and the rescale it treats as automatic, section "Fully
 * Homomorphic Encryption").  The paper is silent on RNS, the NTT, key
 * switching and randomness; the canonical readings taken for those are listed
 * beside each routine.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <stdlib.h>

typedef uint64_t u64;
typedef int64_t i64;
typedef uint32_t u32;
typedef unsigned __int128 u128;

/* ---------------------------------------------------------------- scalars */

u64 orc_mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }

u64 orc_addmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + b) % q); }

u64 orc_submod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + q - (b % q)) % q); }

u64 orc_powmod(u64 b, u64 e, u64 q)
{
    u64 r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = orc_mulmod(r, b, q);
        b = orc_mulmod(b, b, q);
        e >>= 1;
    }
    return r;
}

/* inverse modulo a prime (Fermat) */
u64 orc_invmod(u64 a, u64 q) { return orc_powmod(a, q - 2, q); }

/* [x]_q for a signed integer x, in [0, q) */
u64 orc_reduce_i64(i64 x, u64 q)
{
    if (x >= 0) return (u64)x % q;
    u64 m = (u64)(-(x + 1)) + 1; /* |x| without overflow at INT64_MIN */
    m %= q;
    return m ? q - m : 0;
}

/* Deterministic Miller-Rabin with the first twelve primes as bases; exact for
 * every n < 2^64 (Sorenson & Webster 2015). */
int orc_is_prime(u64 n)
{
    static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    u64 d = n - 1;
    int r = 0;
    while ((d & 1) == 0) { d >>= 1; r++; }
    for (int i = 0; i < 12; i++) {
        u64 x = orc_powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int composite = 1;
        for (int k = 1; k < r; k++) {
            x = orc_mulmod(x, x, n);
            if (x == n - 1) { composite = 0; break; }
        }
        if (composite) return 0;
    }
    return 1;
}

static u32 bitrev(u32 x, u32 bits)
{
    u32 r = 0;
    for (u32 i = 0; i < bits; i++) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}

/* -------------------------------------------------------------------- NTT */

/* fwd[k] = psi^brev(k), inv[k] = psi^-brev(k), k < N (log2 N = logn bits). */
void orc_ntt_tables(u32 logn, u64 q, u64 psi, u64 *fwd, u64 *inv)
{
    u32 n = 1u << logn;
    u64 psi_inv = orc_invmod(psi, q);
    for (u32 k = 0; k < n; k++) {
        u32 e = bitrev(k, logn);
        fwd[k] = orc_powmod(psi, e, q);
        inv[k] = orc_powmod(psi_inv, e, q);
    }
}

/* Negacyclic NTT, output in bit-reversed evaluation order:
 *   out[i] = sum_t a_t * psi^((2*brev(i)+1)*t)  mod q.
 * Radix-2 Cooley-Tukey with the merged psi twiddles (Longa & Naehrig 2016). */
void orc_ntt(u64 *a, u32 logn, u64 q, const u64 *fwd)
{
    u32 n = 1u << logn;
    u32 t = n;
    for (u32 m = 1; m < n; m <<= 1) {
        t >>= 1;
        for (u32 i = 0; i < m; i++) {
            u64 w = fwd[m + i];
            for (u32 j = 2 * i * t; j < 2 * i * t + t; j++) {
                u64 u = a[j];
                u64 v = orc_mulmod(a[j + t], w, q);
                a[j] = orc_addmod(u, v, q);
                a[j + t] = orc_submod(u, v, q);
            }
        }
    }
}

/* Inverse of orc_ntt: Gentleman-Sande with inverse twiddles, then times N^-1. */
void orc_intt(u64 *a, u32 logn, u64 q, const u64 *inv)
{
    u32 n = 1u << logn;
    u32 t = 1;
    for (u32 m = n >> 1; m >= 1; m >>= 1) {
        for (u32 i = 0; i < m; i++) {
            u64 w = inv[m + i];
            for (u32 j = 2 * i * t; j < 2 * i * t + t; j++) {
                u64 u = a[j];
                u64 v = a[j + t];
                a[j] = orc_addmod(u, v, q);
                a[j + t] = orc_mulmod(orc_submod(u, v, q), w, q);
            }
        }
        t <<= 1;
    }
    u64 ninv = orc_invmod(n % q, q);
    for (u32 j = 0; j < n; j++) a[j] = orc_mulmod(a[j], ninv, q);
}

/* ------------------------------------------------------ limb-wise vectors */

void orc_vec_add(const u64 *a, const u64 *b, u64 *out, size_t n, u64 q)
{
    for (size_t i = 0; i < n; i++) out[i] = orc_addmod(a[i], b[i], q);
}

void orc_vec_sub(const u64 *a, const u64 *b, u64 *out, size_t n, u64 q)
{
    for (size_t i = 0; i < n; i++) out[i] = orc_submod(a[i], b[i], q);
}

void orc_vec_neg(const u64 *a, u64 *out, size_t n, u64 q)
{
    for (size_t i = 0; i < n; i++) out[i] = orc_submod(0, a[i], q);
}

void orc_vec_mul(const u64 *a, const u64 *b, u64 *out, size_t n, u64 q)
{
    for (size_t i = 0; i < n; i++) out[i] = orc_mulmod(a[i], b[i], q);
}

void orc_vec_mul_scalar(const u64 *a, u64 c, u64 *out, size_t n, u64 q)
{
    for (size_t i = 0; i < n; i++) out[i] = orc_mulmod(a[i], c % q, q);
}

void orc_vec_reduce_i64(const i64 *x, u64 *out, size_t n, u64 q)
{
    for (size_t i = 0; i < n; i++) out[i] = orc_reduce_i64(x[i], q);
}

/* out = a * b in Z_q[X]/(X^N + 1), via NTT -> pointwise -> inverse NTT. */
void orc_poly_mul(const u64 *a, const u64 *b, u64 *out, u32 logn, u64 q,
                  const u64 *fwd, const u64 *inv, u64 *scratch /* N words */)
{
    u32 n = 1u << logn;
    memcpy(out, a, n * sizeof(u64));
    memcpy(scratch, b, n * sizeof(u64));
    orc_ntt(out, logn, q, fwd);
    orc_ntt(scratch, logn, q, fwd);
    for (u32 i = 0; i < n; i++) out[i] = orc_mulmod(out[i], scratch[i], q);
    orc_intt(out, logn, q, inv);
}

/* Galois automorphism X -> X^g on a coefficient vector (g odd):
 * coefficient t moves to g*t mod 2N, negated when that index is >= N. */
void orc_automorphism(const u64 *a, u64 *out, u32 logn, u64 g, u64 q)
{
    u64 n = 1ull << logn;
    for (u64 t = 0; t < n; t++) {
        u64 e = (u64)(((u128)g * t) % (2 * n));
        if (e < n) out[e] = a[t];
        else out[e - n] = orc_submod(0, a[t], q);
    }
}

/* Fast base conversion without correction (Cheon, Han, Kim, Kim, Song, SAC 2018),
 * with centred remainders: input limbs d_i modulo q_i (i < n_in) of one
 * polynomial; for each target modulus t_o,
 *     y_i = [d_i * Qhat_i^-1]_{q_i} taken in (-q_i/2, q_i/2],
 *     x_o = sum_i y_i * [Qhat_i]_{t_o}  mod t_o,
 * with Qhat_i = prod_{i' != i} q_{i'}.  The integer sum_i y_i Qhat_i is
 * congruent to d modulo Q = prod q_i and lies in (-n_in Q/2, n_in Q/2], so its
 * error against d is e Q with |e| <= n_in/2 and zero mean.  Every constant is
 * formed here from its definition. */
void orc_base_convert(const u64 *in, u32 n_in, const u64 *q_in,
                      u64 *out, u32 n_out, const u64 *q_out, u32 n)
{
    for (u32 o = 0; o < n_out; o++) {
        u64 t = q_out[o];
        for (u32 c = 0; c < n; c++) out[(size_t)o * n + c] = 0;
        for (u32 i = 0; i < n_in; i++) {
            u64 qi = q_in[i];
            u64 qhat_mod_qi = 1 % qi, qhat_mod_t = 1 % t;
            for (u32 k = 0; k < n_in; k++) {
                if (k == i) continue;
                qhat_mod_qi = orc_mulmod(qhat_mod_qi, q_in[k] % qi, qi);
                qhat_mod_t = orc_mulmod(qhat_mod_t, q_in[k] % t, t);
            }
            u64 qhat_inv = orc_invmod(qhat_mod_qi, qi);
            for (u32 c = 0; c < n; c++) {
                u64 y = orc_mulmod(in[(size_t)i * n + c], qhat_inv, qi);
                u64 term;
                if (y <= qi / 2)
                    term = orc_mulmod(y % t, qhat_mod_t, t);
                else  /* y - q_i < 0 */
                    term = orc_submod(0, orc_mulmod((qi - y) % t, qhat_mod_t, t), t);
                u64 *dst = &out[(size_t)o * n + c];
                *dst = orc_addmod(*dst, term, t);
            }
        }
    }
}

/* One limb of the rescale by q_last: r = centred c_last in (-q_last/2, q_last/2),
 * out = (c_i - [r]_{q_i}) * q_last^-1  mod q_i. */
void orc_rescale_limb(const u64 *ci, const u64 *clast, u64 *out, size_t n,
                      u64 qi, u64 qlast)
{
    u64 qinv = orc_invmod(qlast % qi, qi);
    for (size_t t = 0; t < n; t++) {
        i64 r = (clast[t] > qlast / 2) ? -(i64)(qlast - clast[t]) : (i64)clast[t];
        u64 rq = orc_reduce_i64(r, qi);
        out[t] = orc_mulmod(orc_submod(ci[t], rq, qi), qinv, qi);
    }
}

/* --------------------------------------------------------------- ChaCha20 */

static u32 rotl32(u32 x, int n) { return (x << n) | (x >> (32 - n)); }

static void quarter(u32 *s, int a, int b, int c, int d)
{
    s[a] += s[b]; s[d] ^= s[a]; s[d] = rotl32(s[d], 16);
    s[c] += s[d]; s[b] ^= s[c]; s[b] = rotl32(s[b], 12);
    s[a] += s[b]; s[d] ^= s[a]; s[d] = rotl32(s[d], 8);
    s[c] += s[d]; s[b] ^= s[c]; s[b] = rotl32(s[b], 7);
}

/* RFC 8439 section 2.1 quarter round on four words (exported for its test vector). */
void orc_chacha_quarter(u32 *abcd)
{
    quarter(abcd, 0, 1, 2, 3);
}

/* RFC 8439 section 2.3 block function: 16 output words (state after 20 rounds
 * plus the input state). */
void orc_chacha20_block(const u32 *key8, u32 counter, const u32 *nonce3, u32 *out16)
{
    u32 init[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u,
                    key8[0], key8[1], key8[2], key8[3],
                    key8[4], key8[5], key8[6], key8[7],
                    counter, nonce3[0], nonce3[1], nonce3[2]};
    u32 s[16];
    memcpy(s, init, sizeof s);
    for (int r = 0; r < 10; r++) {
        quarter(s, 0, 4, 8, 12);
        quarter(s, 1, 5, 9, 13);
        quarter(s, 2, 6, 10, 14);
        quarter(s, 3, 7, 11, 15);
        quarter(s, 0, 5, 10, 15);
        quarter(s, 1, 6, 11, 12);
        quarter(s, 2, 7, 8, 13);
        quarter(s, 3, 4, 9, 14);
    }
    for (int i = 0; i < 16; i++) out16[i] = s[i] + init[i];
}

/* Keystream words for (seed, purpose, object): the ChaCha20 key is the 256-bit
 * seed as 32 little-endian bytes (seed4[0] holds bits 0..63); nonce = purpose
 * (u32 LE) || object (u64 LE); block counter from 0; 64-bit word w is bytes
 * 8w..8w+7 of the stream, little-endian. */
void orc_stream_words(const u64 *seed4, u32 purpose, u64 obj, u64 first, size_t count, u64 *out)
{
    u32 key[8];
    for (int i = 0; i < 4; i++) {
        key[2 * i] = (u32)seed4[i];
        key[2 * i + 1] = (u32)(seed4[i] >> 32);
    }
    u32 nonce[3] = {purpose, (u32)obj, (u32)(obj >> 32)};
    u32 blk[16];
    u64 cur = ~0ull;
    for (size_t k = 0; k < count; k++) {
        u64 w = first + k;
        u64 b = w / 8;
        if (b != cur) {
            orc_chacha20_block(key, (u32)b, nonce, blk);
            cur = b;
        }
        u32 j = (u32)(w % 8);
        out[k] = (u64)blk[2 * j] | ((u64)blk[2 * j + 1] << 32);
    }
}

/* Ternary sample from one stream word: floor(3w / 2^64) - 1 in {-1, 0, 1};
 * coefficient t uses word t. */
void orc_sample_ternary(const u64 *seed, u32 purpose, u64 obj, size_t n, i64 *out)
{
    u64 *w = (u64 *)malloc(n * sizeof(u64));
    orc_stream_words(seed, purpose, obj, 0, n, w);
    for (size_t t = 0; t < n; t++) out[t] = (i64)(((u128)w[t] * 3) >> 64) - 1;
    free(w);
}

/* Discrete Gaussian by cumulative table: coefficient t uses word t; bit 63 is
 * the sign, the low 63 bits r give |x| = min{k : r < T[k]} (T has 20 entries,
 * T[19] = 2^63); a zero magnitude ignores the sign. */
void orc_sample_gauss(const u64 *seed, u32 purpose, u64 obj, size_t n, const u64 *cdt, i64 *out)
{
    u64 *w = (u64 *)malloc(n * sizeof(u64));
    orc_stream_words(seed, purpose, obj, 0, n, w);
    for (size_t t = 0; t < n; t++) {
        u64 r = w[t] & 0x7fffffffffffffffull;
        i64 k = 0;
        while (k < 19 && r >= cdt[k]) k++;
        out[t] = ((w[t] >> 63) && k) ? -k : k;
    }
    free(w);
}

/* Uniform sample mod q for limb `limb`: coefficient t takes stream words
 * 2(limb*N + t) (low half) and 2(limb*N + t) + 1 (high half) of a 128-bit W,
 * and the value is floor(W * q / 2^128), computed as a 192-bit product. */
void orc_sample_uniform(const u64 *seed, u32 purpose, u64 obj, u32 limb, u32 logn, u64 q, u64 *out)
{
    u64 n = 1ull << logn;
    u64 *w = (u64 *)malloc(2 * n * sizeof(u64));
    orc_stream_words(seed, purpose, obj, 2 * (u64)limb * n, 2 * n, w);
    for (u64 t = 0; t < n; t++) {
        u128 lo = (u128)w[2 * t] * q;                 /* bits 0..127 of W_lo * q */
        u128 hi = (u128)w[2 * t + 1] * q + (lo >> 64); /* bits 64..191 of W * q  */
        out[t] = (u64)(hi >> 64);
    }
    free(w);
}
