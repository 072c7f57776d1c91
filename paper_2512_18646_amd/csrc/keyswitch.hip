// Hybrid key switching (Han & Ki, CT-RSA 2020) on gfx950: ModUp by fast base
// conversion, inner product with the switching key, ModDown.
//
// Base conversion (Cheon, Han, Kim, Kim, Song, SAC 2018, without correction,
// centred remainders): for input limbs d_i mod q_i (i in a digit) and every
// target modulus t,
//     y_i = [d_i * Qhat_i^-1]_{q_i} (taken in (-q_i/2, q_i/2]),
//     x_t = sum_i y_i [Qhat_i]_t = sum_i y_i' [Qhat_i]_t + n_neg [-Q]_t  (mod t)
// where y_i' is the [0, q_i) representative and n_neg counts the y_i above
// q_i / 2 (each contributes -q_i Qhat_i = -Q).  One thread per coefficient
// keeps the <= 16 inputs in registers and streams the targets; the 128-bit
// dot product is reduced once per target.
//
// The same contraction on the matrix cores, exactly: every y_i (< 2^60) and
// every constant W (< 2^61) is written in balanced base 256, eight signed
// digits in [-128, 127], so that sum_i y_i W = sum_c 2^(8c) S_c with
// S_c = sum_{i, a + b = c} y_{i,a} W_{i,b} an int8 dot product (|S_c| < 2^21).
// One v_mfma_i32_16x16x32_i8 takes 4 inputs x 8 digits on K, 16 coefficients
// on N and (4 targets x 4 values of c) on M; four such tiles give a lane all
// sixteen S_c of one (target, coefficient), which it shifts into the exact
// 128-bit sum and reduces once.  The n_neg term rides along as one more input
// whose only digit is n_neg.  Which kernel runs is timed once per table.
//
// Inner product: every extended limb e reads the beta digits of X (through the
// Galois permutation for rotations) and the key limbs b_j, a_j once; the
// batched form keeps the key values in registers and loops over ciphertexts
// that share the key, so the key streams from HBM once per batch.
#include "vr_ops.h"

namespace vr {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxIn = 16;


typedef int v4i __attribute__((ext_vector_type(4)));

// balanced base-256 digits of x < 2^63 as eight signed bytes:
// x = sum_a d_a 256^a with byte a = d_a
__host__ __device__ __forceinline__ u64 balanced_bytes(u64 x)
{
    const u64 h = 0x8080808080808080ull;
    return (x + h) ^ h;
}

struct ConvArgs {
    const u64* in;            // input limb i: in + poly * in_stride + i * N
    u64 in_stride;
    u64* out;                 // output o: out + poly * out_stride + slot(o) * N
    u64 out_stride;
    u32 skip_at, skip_len;    // slot(o) = o < skip_at ? o : o + skip_len
    const u64* tab;
    u32 n_in, n_out;
    u32 log_n;
    const ModQ* mq;
    u32 o_lo = 0, o_hi = 0xffffffffu;   // the targets the integer and FP64 kernels make
};
VR_KERNEL_ARG(ConvArgs);

constexpr int kMaxOut = 48;

// Constants are staged in LDS per block (qhat [n_out][n_in] transposed so one
// output's row is contiguous, plus q, 2^64 mod q and the Shoup companions of
// each target), then every thread converts one coefficient.
__global__ __launch_bounds__(kThreads) void k_base_convert(ConvArgs a)
{
    __shared__ u64 s_qhat[kMaxIn * kMaxOut];
    __shared__ u64 s_out[kMaxOut * 5];   // q, r64, r64_s, one_s, negq
    const u32 n = 1u << a.log_n;
    const u32 poly = blockIdx.y;
    const u64* qinv = a.tab;
    const u64* qinv_s = a.tab + a.n_in;
    const u64* qhat = a.tab + 2 * a.n_in;
    const u64* negq = qhat + (size_t)a.n_in * a.n_out;
    const u64* in_mod = negq + a.n_out;
    const u64* out_mod = in_mod + a.n_in;
    for (u32 e = threadIdx.x; e < a.n_in * a.n_out; e += kThreads) {
        u32 i = e / a.n_out, o = e - i * a.n_out;
        s_qhat[o * a.n_in + i] = qhat[e];
    }
    for (u32 o = threadIdx.x; o < a.n_out; o += kThreads) {
        const ModQ& m = a.mq[out_mod[o]];
        s_out[5 * o] = m.q;
        s_out[5 * o + 1] = m.r64;
        s_out[5 * o + 2] = m.r64_s;
        s_out[5 * o + 3] = m.one_s;
        s_out[5 * o + 4] = negq[o];
    }
    __syncthreads();
    const u32 t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    const u64* in = a.in + (size_t)poly * a.in_stride;
    u64* out = a.out + (size_t)poly * a.out_stride;

    u64 y[kMaxIn];
    u64 n_neg = 0;
#pragma unroll
    for (int i = 0; i < kMaxIn; i++) {
        if (i < (int)a.n_in) {
            u64 q = a.mq[in_mod[i]].q;
            u64 v = shoup(in[(size_t)i * n + t], qinv[i], qinv_s[i], q);
            n_neg += v > (q >> 1) ? 1 : 0;
            y[i] = v;
        }
    }
    const u32 o_end = min(a.o_hi, a.n_out);
#pragma unroll 2
    for (u32 o = a.o_lo; o < o_end; o++) {
        const u64* c = s_out + 5 * o;
        u64 hi = 0, lo = 0;
        mac128(hi, lo, n_neg, c[4]);
        const u64* qh = s_qhat + o * a.n_in;
#pragma unroll
        for (int i = 0; i < kMaxIn; i++)
            if (i < (int)a.n_in) mac128(hi, lo, y[i], qh[i]);
        const u64 q = c[0];
        u64 r = shoup_lazy(hi, c[1], c[2], q) + shoup_lazy(lo, 1, c[3], q);
        r = csub(r, 2 * q);
        u32 slot = o < a.skip_at ? o : o + a.skip_len;
        out[(size_t)slot * n + t] = csub(r, q);
    }
}

// The same conversion in FP64 for targets t < 2^51 (the 128-bit integer form
// above for wider targets): y_i centred, held exactly as a double when
// q_i < 2^51; a 60-bit first input (q_0 in digit 0) is held as halves
// y = yh 2^30 + yl (yl in [0, 2^30)).  The constants are balanced mod t,
// [Qhat_i]_t (and [2^30 Qhat_0]_t), in rows zero-padded to kMaxIn inputs, so
// the product loop has no branches and its wave-uniform constant loads issue
// together.  Each product is formed exactly (fmulmod; |y W / t| <= 2^49
// keeps it within 0.69 t of zero) and the sum is reduced every four products,
// staying below 3.3 t < 2^53.
struct ConvFp {
    const double* w;   // [n_out][kMaxIn][2]: balanced [Qhat_i]_t, [2^30 Qhat_i]_t
    const double* t;   // [n_out][2]: t, 1 / t
};
VR_KERNEL_ARG(ConvFp);

constexpr double kTwo51 = 2251799813685248.0;

// Up to ten inputs the kernel is held to 5 waves per SIMD (ten spill a few
// registers; measured faster than 4 waves without the spill).
template <int NI, bool W0>
__global__ __launch_bounds__(kThreads, NI <= 10 ? 5 : 1) void k_base_convert_fp(ConvArgs a, ConvFp f)
{
    const u32 n = 1u << a.log_n;
    const u32 poly = blockIdx.y;
    const u64* qinv = a.tab;
    const u64* qinv_s = a.tab + a.n_in;
    const u64* qhat = a.tab + 2 * a.n_in;
    const u64* negq = qhat + (size_t)a.n_in * a.n_out;
    const u64* in_mod = negq + a.n_out;
    const u64* out_mod = in_mod + a.n_in;
    const u32 t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    const u64* in = a.in + (size_t)poly * a.in_stride;
    u64* out = a.out + (size_t)poly * a.out_stride;

    u64 x[NI];
#pragma unroll
    for (int i = 0; i < NI; i++)
        if (i < (int)a.n_in) x[i] = in[(size_t)i * n + t];
    double yl[NI], yh0 = 0.0;
    u64 qin[NI];   // input moduli, read once (the integer form for wide targets needs them)
#pragma unroll
    for (int i = 0; i < NI; i++) {
        yl[i] = 0.0;
        qin[i] = 0;
        if (i < (int)a.n_in) {
            const u64 q = a.mq[in_mod[i]].q;
            qin[i] = q;
            const u64 v = shoup(x[i], qinv[i], qinv_s[i], q);
            if (W0 && i == 0) {
                const i64 y = v > (q >> 1) ? (i64)v - (i64)q : (i64)v;
                yh0 = (double)(int)(y >> 30);
                yl[0] = (double)(u32)(y & ((1ll << 30) - 1));
            } else {
                yl[i] = to_bal(v, q, (double)q);
            }
        }
    }
    // target o + 1's constants are loaded while target o is summed
    double wc[NI], wh = 0.0, tc[2];
#pragma unroll
    for (int i = 0; i < NI; i++) wc[i] = f.w[(size_t)a.o_lo * kMaxIn * 2 + 2 * i];
    if (W0) wh = f.w[(size_t)a.o_lo * kMaxIn * 2 + 1];
    tc[0] = f.t[2 * a.o_lo];
    tc[1] = f.t[2 * a.o_lo + 1];
    const u32 o_end = min(a.o_hi, a.n_out);
    for (u32 o = a.o_lo; o < o_end; o++) {
        const double td = tc[0], tinv = tc[1];
        double w[NI], w1 = wh;
#pragma unroll
        for (int i = 0; i < NI; i++) w[i] = wc[i];
        if (o + 1 < o_end) {
            const double* wn = f.w + (size_t)(o + 1) * kMaxIn * 2;
#pragma unroll
            for (int i = 0; i < NI; i++) wc[i] = wn[2 * i];
            if (W0) wh = wn[1];
            tc[0] = f.t[2 * (o + 1)];
            tc[1] = f.t[2 * (o + 1) + 1];
        }
        u64 r;
        if (td < kTwo51) {
            double acc = 0.0;
            int since = 0;   // products since the last reduction (compile time)
#pragma unroll
            for (int i = 0; i < NI; i++) {
                acc += fmulmod(yl[i], w[i], td, tinv);
                since++;
                if (W0 && i == 0) {
                    acc += fmulmod(yh0, w1, td, tinv);
                    since++;
                }
                if (since >= 4 && i + 1 < NI) {
                    acc = fbal(acc, td, tinv);
                    since = 0;
                }
            }
            r = to_canon(acc, td, tinv);
        } else {
            u64 hi = 0, lo = 0, nn = 0;
#pragma unroll
            for (int i = 0; i < NI; i++) {
                if (i < (int)a.n_in) {
                    const u64 q = qin[i];
                    const i64 y = (W0 && i == 0) ? ((i64)(int)yh0 << 30) + (i64)(u32)yl[0] : (i64)yl[i];
                    nn += y < 0 ? 1 : 0;
                    mac128(hi, lo, (u64)(y < 0 ? y + (i64)q : y), qhat[(size_t)i * a.n_out + o]);
                }
            }
            mac128(hi, lo, nn, negq[o]);
            const ModQ& m = a.mq[out_mod[o]];
            const u64 tq = m.q;
            r = shoup_lazy(hi, m.r64, m.r64_s, tq) + shoup_lazy(lo, 1, m.one_s, tq);
            r = csub(csub(r, 2 * tq), tq);
        }
        const u32 slot = o < a.skip_at ? o : o + a.skip_len;
        out[(size_t)slot * n + t] = r;
    }
}

constexpr u32 kMfmaCoef = 256;    // coefficients per block: 4 waves x 4 tiles of 16
constexpr u32 kDigitRow = 264;    // LDS row pitch of the digit words (padded)

__global__ __launch_bounds__(256) void k_base_convert_mfma(ConvArgs a, const u64* wt, u32 steps,
                                                            u32 groups, u32 n_polys)
{
    extern __shared__ u64 lds[];
    const u32 tw = groups * 4 * steps * 64;
    u64* s_wt = lds;                  // [groups][4][steps][64]
    u64* s_d = lds + tw;              // [4 * steps][kDigitRow]
    for (u32 e = threadIdx.x; e < tw; e += 256) s_wt[e] = wt[e];
    const u32 n = 1u << a.log_n;
    const u64* qinv = a.tab;
    const u64* qinv_s = a.tab + a.n_in;
    const u64* in_mod = a.tab + 2 * a.n_in + (size_t)a.n_in * a.n_out + a.n_out;
    const u64* out_mod = in_mod + a.n_in;
    const u32 base = blockIdx.x * kMfmaCoef;
    const u32 lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const u32 g = lane >> 4, col = lane & 15;
    for (u32 poly = blockIdx.y; poly < n_polys; poly += gridDim.y) {
        // digit words of this block's coefficients: row i = input i, row n_in = n_neg
        const u64* in = a.in + (size_t)poly * a.in_stride;
        const u32 t = base + threadIdx.x;
        u32 n_neg = 0;
        for (u32 i = 0; i < 4 * steps; i++) {
            u64 w = 0;
            if (i < a.n_in && t < n) {
                const u64 q = a.mq[in_mod[i]].q;
                const u64 v = shoup(in[(size_t)i * n + t], qinv[i], qinv_s[i], q);
                n_neg += v > (q >> 1) ? 1 : 0;
                w = balanced_bytes(v);
            }
            s_d[i * kDigitRow + threadIdx.x] = w;
        }
        s_d[a.n_in * kDigitRow + threadIdx.x] = n_neg;
        __syncthreads();
        u64* out = a.out + (size_t)poly * a.out_stride;
        for (u32 u = 0; u < 4; u++) {
            const u32 nl = wave * 64 + u * 16 + col;
            const u32 coef = base + nl;
            long b[4];
#pragma unroll
            for (u32 s = 0; s < 4; s++) b[s] = s < steps ? (long)s_d[(4 * s + g) * kDigitRow + nl] : 0;
            for (u32 G = 0; G < groups; G++) {
                i64 P[4];
#pragma unroll
                for (u32 m = 0; m < 4; m++) {
                    v4i acc = {0, 0, 0, 0};
                    const u64* w = s_wt + (size_t)(G * 4 + m) * steps * 64 + lane;
#pragma unroll
                    for (u32 s = 0; s < 4; s++)
                        if (s < steps)
                            acc = __builtin_amdgcn_mfma_i32_16x16x32_i8((long)w[s * 64], b[s], acc, 0, 0, 0);
                    // rows 4g + r of tile m are c = 4m + r of target 4G + g
                    P[m] = (i64)acc[0] + ((i64)acc[1] << 8) + ((i64)acc[2] << 16) + ((i64)acc[3] << 24);
                }
                // V = sum_m P[m] 2^(32 m), exact in two's complement 128 bits
                u64 lo = (u64)P[0], hi = (u64)(P[0] >> 63);
                const u64 x1 = (u64)P[1] << 32;
                lo += x1;
                hi += (u64)(P[1] >> 32) + (lo < x1 ? 1 : 0);
                hi += (u64)P[2] + ((u64)P[3] << 32);
                const u32 o = G * 4 + g;
                if (o < a.n_out && coef < n) {
                    const ModQ& mq = a.mq[out_mod[o]];
                    const u32 slot = o < a.skip_at ? o : o + a.skip_len;
                    out[(size_t)slot * n + coef] = reduce128(hi, lo, mq);
                }
            }
        }
        __syncthreads();
    }
}

// One block = 256 consecutive source words of extended limb e.  With a Galois
// element g != 1 output t reads source sigma(t); the block's sources form one
// aligned 256-word chunk whose outputs t = sigma^-1(s) (g_inv = g^-1 mod 2N)
// form another (the top index bits of the bit-reversed order map among
// themselves under X -> X^g).  So each thread loads its source words
// coalesced, takes the key at its output index (loaded once per block, the
// key being shared by every ciphertext of the batch), and writes its output
// within that chunk: no staging and no barrier per ciphertext.  The next
// ciphertext's digits are loaded while the current one is summed.
//
// FP = the launch covers limbs whose moduli are below 2^51: FP64 products
// with key and inputs balanced, each product within 0.75 q, the sums reduced
// every four digits (below 3.5 q < 2^53).  Otherwise 128-bit integer sums.
// The launch covers the extended limbs of up to kMaxRuns runs [b, b + len),
// blockIdx.y enumerating them in order.
constexpr int kMaxRuns = 4;
struct LimbRuns {
    u32 b[kMaxRuns], len[kMaxRuns];
    u32 o[kMaxRuns];   // output position (limb of U) of each run's first limb
};
VR_KERNEL_ARG(LimbRuns);

// Up to two rotation steps per launch (NS): step k has its key, its output
// slab and g_inv; every digit word (and the c0 word of the fold) is read
// once for both, and each step writes its own permuted chunk.
struct KsSteps {
    const u64* key[2];
    u64* U[2];
    u32 g_inv[2];
};
VR_KERNEL_ARG(KsSteps);

template <int MAXB, bool FP, int NS>
__global__ __launch_bounds__(kThreads) void k_ks_inner(const u64* X, u64 x_stride, const u64* D,
                                                      u64 d_stride, u32 n_ct, KsSteps st, u32 nmod,
                                                      u32 level, u32 next, u32 beta, u32 alpha, u32 L,
                                                      u32 log_n, u64 u_stride, const ModQ* mq, LimbRuns runs,
                                                      const u64* F, u64 f_stride, const ulonglong2* pmod,
                                                      u32 u_limbs)
{
    const u32 n = 1u << log_n;
    const u32 s = blockIdx.x * kThreads + threadIdx.x;
    if (s >= n) return;
    u32 e = blockIdx.y, r = 0;
    while (r + 1 < kMaxRuns && e >= runs.len[r]) e -= runs.len[r++];
    const u32 pos = runs.o[r] + e;   // limb of U this block writes
    e += runs.b[r];
    const u32 mod = e <= level ? e : L + 1 + (e - level - 1);
    const ModQ m = mq[mod];
    u32 t[NS];
#pragma unroll
    for (int k = 0; k < NS; k++) t[k] = st.g_inv[k] != 1 ? galois_src(s, st.g_inv[k], log_n) : s;
    // blockIdx.z splits the ciphertexts into groups so small rings still fill the chip
    const u32 per = (n_ct + gridDim.z - 1) / gridDim.z;
    const u32 c_lo = blockIdx.z * per, c_hi = min(n_ct, c_lo + per);
    if (c_lo >= c_hi) return;
    // the digit owning limb e (a Q limb) takes it from the ModUp input
    const u32 own = e <= level ? e / alpha : 0xffffffffu;
    auto load = [&](u32 c, u64 (&xv)[MAXB]) {
        const u64* xc = X + (size_t)c * x_stride + (size_t)e * n + s;
        const u64* dc = D + (size_t)c * d_stride + (size_t)(e <= level ? e : 0) * n + s;
#pragma unroll
        for (int j = 0; j < MAXB; j++)
            if (j < (int)beta) xv[j] = own == (u32)j ? dc[0] : xc[(size_t)j * next * n];
    };
    if constexpr (FP) {
        const double qd = (double)m.q, qinv = 1.0 / qd;
        const double pf = F && e <= level ? to_bal(pmod[mod].x, m.q, qd) : 0.0;
        double fb[NS][MAXB], fa[NS][MAXB];
#pragma unroll
        for (int k = 0; k < NS; k++)
#pragma unroll
            for (int j = 0; j < MAXB; j++) {
                if (j < (int)beta) {
                    fb[k][j] = to_bal(st.key[k][((size_t)(2 * j) * nmod + mod) * n + t[k]], m.q, qd);
                    fa[k][j] = to_bal(st.key[k][((size_t)(2 * j + 1) * nmod + mod) * n + t[k]], m.q, qd);
                }
            }
        u64 xv[MAXB], xn[MAXB];
        load(c_lo, xv);
        for (u32 c = c_lo; c < c_hi; c++) {
            if (c + 1 < c_hi) load(c + 1, xn);
            double x[MAXB];
#pragma unroll
            for (int j = 0; j < MAXB; j++)
                if (j < (int)beta) x[j] = to_bal(xv[j], m.q, qd);
            // + P sigma_g(c0): c0 read where X is, stored where U is
            const double fc = F && e <= level
                                  ? fmulmod(to_bal(F[(size_t)c * f_stride + (size_t)e * n + s], m.q, qd), pf, qd, qinv)
                                  : 0.0;
#pragma unroll
            for (int k = 0; k < NS; k++) {
                double s0 = 0, s1 = 0;
#pragma unroll
                for (int j = 0; j < MAXB; j++) {
                    if (j < (int)beta) {
                        s0 += fmulmod(x[j], fb[k][j], qd, qinv);
                        s1 += fmulmod(x[j], fa[k][j], qd, qinv);
                        if ((j & 3) == 3) {
                            s0 = fbal(s0, qd, qinv);
                            s1 = fbal(s1, qd, qinv);
                        }
                    }
                }
                s0 += fc;
                u64* u = st.U[k] + (size_t)c * u_stride + (size_t)pos * n + t[k];
                u[0] = to_canon(s0, qd, qinv);
                u[(size_t)u_limbs * n] = to_canon(s1, qd, qinv);
            }
#pragma unroll
            for (int j = 0; j < MAXB; j++) xv[j] = xn[j];
        }
    } else {
        u64 kb[NS][MAXB], ka[NS][MAXB];
#pragma unroll
        for (int k = 0; k < NS; k++)
#pragma unroll
            for (int j = 0; j < MAXB; j++) {
                if (j < (int)beta) {
                    kb[k][j] = st.key[k][((size_t)(2 * j) * nmod + mod) * n + t[k]];
                    ka[k][j] = st.key[k][((size_t)(2 * j + 1) * nmod + mod) * n + t[k]];
                }
            }
        for (u32 c = c_lo; c < c_hi; c++) {
            u64 xv[MAXB];
            load(c, xv);
            const u64 fw = F && e <= level ? F[(size_t)c * f_stride + (size_t)e * n + s] : 0;
#pragma unroll
            for (int k = 0; k < NS; k++) {
                u64 h0 = 0, l0 = 0, h1 = 0, l1 = 0;
#pragma unroll
                for (int j = 0; j < MAXB; j++) {
                    if (j < (int)beta) {
                        mac128(h0, l0, xv[j], kb[k][j]);
                        mac128(h1, l1, xv[j], ka[k][j]);
                    }
                }
                if (F && e <= level) mac128(h0, l0, fw, pmod[mod].x);
                u64* u = st.U[k] + (size_t)c * u_stride + (size_t)pos * n + t[k];
                u[0] = reduce128(h0, l0, m);
                u[(size_t)u_limbs * n] = reduce128(h1, l1, m);
            }
        }
    }
}

// out_k = (U_k - Y_k) e_i (+ add_k b_i, or + add_k when bm is null), k = 0,
// 1; limb i < nq, (e_i, b_i) = (cm[i], bm[i]) with Shoup companions
__global__ __launch_bounds__(kThreads) void k_moddown_finish(
    const u64* U, u64 u_stride, const u64* Y, u32 nq, u32 next, u32 log_n, u64* out0, u64* out1,
    u64 out_stride, const u64* add0, u32 add0_g, const u64* add1, u64 add_stride, const ModQ* mq,
    const ulonglong2* cm, const ulonglong2* bm)
{
    const u32 n = 1u << log_n;
    const u32 t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    const u32 i = blockIdx.y % nq;
    const u32 c = blockIdx.y / nq;
    const u64 q = mq[i].q;
    const ulonglong2 e = cm[i];
    const u64* u = U + (size_t)c * u_stride + (size_t)i * n + t;
    const u64* y = Y + ((size_t)c * 2 * nq + i) * n + t;
    u64 r0 = shoup(u[0] + q - y[0], e.x, e.y, q);
    u64 r1 = shoup(u[(size_t)next * n] + q - y[(size_t)nq * n], e.x, e.y, q);
    if (add0) {
        u32 src = add0_g == 1 ? t : galois_src(t, add0_g, log_n);
        u64 b = add0[(size_t)c * add_stride + (size_t)i * n + src];
        r0 = add_mod(r0, bm ? shoup(b, bm[i].x, bm[i].y, q) : b, q);
    }
    if (add1) {
        u64 b = add1[(size_t)c * add_stride + (size_t)i * n + t];
        r1 = add_mod(r1, bm ? shoup(b, bm[i].x, bm[i].y, q) : b, q);
    }
    out0[(size_t)c * out_stride + (size_t)i * n + t] = r0;
    out1[(size_t)c * out_stride + (size_t)i * n + t] = r1;
}

// Fold of P c into the q_l limb before a ModDown by P q_l: u += [P]_{q_l} c
// on limb q_l of both components of every ciphertext (u, c0, c1 point at
// that limb).
__global__ __launch_bounds__(kThreads) void k_fold_pc(u64* U, u64 u_stride, u64 u_comp, const u64* c0,
                                                      const u64* c1, u64 c_stride, u64 pm, u64 pm_s, u64 q,
                                                      u32 n)
{
    const u32 t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    const u32 ct = blockIdx.y >> 1, j = blockIdx.y & 1;
    u64* u = U + (size_t)ct * u_stride + (size_t)j * u_comp + t;
    const u64 c = (j ? c1 : c0)[(size_t)ct * c_stride + t];
    *u = add_mod(*u, shoup(c, pm, pm_s, q), q);
}

u64 powmod_h(u64 b, u64 e, u64 q)
{
    u64 r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = (u64)((u128)r * b % q);
        b = (u64)((u128)b * b % q);
        e >>= 1;
    }
    return r;
}

// Builds the constant table for converting from moduli `in` to moduli `out`
// (indices into ctx->mod).
ConvTable build_table(vr_context* ctx, const std::vector<u32>& in, const std::vector<u32>& out)
{
    ConvTable tb;
    tb.n_in = (u32)in.size();
    tb.n_out = (u32)out.size();
    if (tb.n_in > (u32)kMaxIn) throw Error(VR_EINVAL, "base conversion: too many input moduli");
    if (tb.n_out > (u32)kMaxOut) throw Error(VR_EINVAL, "base conversion: too many output moduli");
    std::vector<u64> h;
    h.resize(2 * tb.n_in + (size_t)tb.n_in * tb.n_out + tb.n_out + tb.n_in + tb.n_out);
    u64* qinv = h.data();
    u64* qinv_s = qinv + tb.n_in;
    u64* qhat = qinv_s + tb.n_in;
    u64* negq = qhat + (size_t)tb.n_in * tb.n_out;
    u64* in_mod = negq + tb.n_out;
    u64* out_mod = in_mod + tb.n_in;
    for (u32 i = 0; i < tb.n_in; i++) {
        u64 qi = ctx->mod[in[i]];
        u64 prod = 1;
        for (u32 k = 0; k < tb.n_in; k++)
            if (k != i) prod = (u64)((u128)prod * (ctx->mod[in[k]] % qi) % qi);
        qinv[i] = powmod_h(prod, qi - 2, qi);
        qinv_s[i] = shoup_companion(qinv[i], qi);
        for (u32 o = 0; o < tb.n_out; o++) {
            u64 to = ctx->mod[out[o]];
            u64 p = 1;
            for (u32 k = 0; k < tb.n_in; k++)
                if (k != i) p = (u64)((u128)p * (ctx->mod[in[k]] % to) % to);
            qhat[(size_t)i * tb.n_out + o] = p;
        }
        in_mod[i] = in[i];
    }
    for (u32 o = 0; o < tb.n_out; o++) {
        u64 to = ctx->mod[out[o]];
        u64 p = 1;
        for (u32 k = 0; k < tb.n_in; k++) p = (u64)((u128)p * (ctx->mod[in[k]] % to) % to);
        negq[o] = p ? to - p : 0;
        out_mod[o] = out[o];
    }
    tb.words = h.size();
    VR_HIP(hipMalloc(&tb.dev, tb.words * sizeof(u64)));
    VR_HIP(hipMemcpy(tb.dev, h.data(), tb.words * sizeof(u64), hipMemcpyHostToDevice));
    // matrix-core table: lane l of (group G, tile m, step s) holds row
    // rho = l % 16 (target 4G + rho / 4, c = 4m + rho % 4) and inputs
    // i = 4s + l / 16; byte a is digit c - a of that input's constant
    tb.steps = (tb.n_in + 1 + 3) / 4;
    tb.groups = (tb.n_out + 3) / 4;
    std::vector<u64> wt((size_t)tb.groups * 4 * tb.steps * 64, 0);
    for (u32 G = 0; G < tb.groups; G++)
        for (u32 m = 0; m < 4; m++)
            for (u32 s = 0; s < tb.steps; s++)
                for (u32 l = 0; l < 64; l++) {
                    const u32 rho = l & 15, o = 4 * G + (rho >> 2), c = 4 * m + (rho & 3);
                    const u32 i = 4 * s + (l >> 4);
                    if (o >= tb.n_out || i > tb.n_in) continue;
                    const u64 W = i < tb.n_in ? qhat[(size_t)i * tb.n_out + o] : negq[o];
                    const u64 e = balanced_bytes(W);
                    u64 word = 0;
                    for (u32 aa = 0; aa < 8; aa++) {
                        const int b = (int)c - (int)aa;
                        if (b >= 0 && b < 8) word |= ((e >> (8 * b)) & 0xff) << (8 * aa);
                    }
                    wt[(((size_t)G * 4 + m) * tb.steps + s) * 64 + l] = word;
                }
    VR_HIP(hipMalloc(&tb.wt, wt.size() * sizeof(u64)));
    VR_HIP(hipMemcpy(tb.wt, wt.data(), wt.size() * sizeof(u64), hipMemcpyHostToDevice));
    // FP64 form: balanced [Qhat_i]_t and [2^30 Qhat_i]_t per (target, input),
    // rows padded with zeros to kMaxIn inputs, then (t, 1/t) per target;
    // entries of targets >= 2^51 are unused
    std::vector<double> wf((size_t)tb.n_out * kMaxIn * 2 + (size_t)tb.n_out * 2, 0.0);
    double* wt_t = wf.data() + (size_t)tb.n_out * kMaxIn * 2;
    tb.wide = 0;
    for (u32 i = 0; i < tb.n_in; i++)
        if (ctx->mod[in[i]] >= (1ull << 51)) tb.wide |= 1u << i;
    tb.wide_out = 0;
    for (u32 o = 0; o < tb.n_out; o++)
        if (ctx->mod[out[o]] >= (1ull << 51)) tb.wide_out |= o < 32 ? 1u << o : 0x80000000u;
    for (u32 o = 0; o < tb.n_out; o++) {
        const u64 to = ctx->mod[out[o]];
        wt_t[2 * o] = (double)to;
        wt_t[2 * o + 1] = 1.0 / (double)to;
        if (to >= (1ull << 51)) continue;
        auto bal = [to](u64 v) { return v > to / 2 ? -(double)(to - v) : (double)v; };
        for (u32 i = 0; i < tb.n_in; i++) {
            const u64 W = qhat[(size_t)i * tb.n_out + o];
            wf[((size_t)o * kMaxIn + i) * 2] = bal(W);
            wf[((size_t)o * kMaxIn + i) * 2 + 1] = bal((u64)(((u128)W << 30) % to));
        }
    }
    VR_HIP(hipMalloc(&tb.wf, wf.size() * sizeof(double)));
    VR_HIP(hipMemcpy(tb.wf, wf.data(), wf.size() * sizeof(double), hipMemcpyHostToDevice));
    tb.choice = std::make_shared<std::atomic<int>>(-1);
    return tb;
}

const ConvTable& modup_table(vr_context* ctx, u32 level, u32 j)
{
    std::lock_guard<std::mutex> g(ctx->mu);
    auto key = std::make_pair((int)level, (int)j);
    auto it = ctx->modup_tables.find(key);
    if (it != ctx->modup_tables.end()) return it->second;
    u32 lo = j * ctx->alpha, hi = std::min((j + 1) * ctx->alpha, level + 1);
    std::vector<u32> in, out;
    for (u32 i = lo; i < hi; i++) in.push_back(i);
    u32 next = level + 1 + ctx->K;
    for (u32 e = 0; e < next; e++)
        if (e < lo || e >= hi) out.push_back(ctx->ext_mod(e, level));
    return ctx->modup_tables[key] = build_table(ctx, in, out);
}

// digit j of `level` to the extended limbs [e0, e1) and then [e2, e3) (none
// of them its own; e2 = e3 for one run)
const ConvTable& modup_range_table(vr_context* ctx, u32 level, u32 j, u32 e0, u32 e1, u32 e2 = 0, u32 e3 = 0)
{
    std::lock_guard<std::mutex> g(ctx->mu);
    const std::array<int, 6> key{(int)level, (int)j, (int)e0, (int)e1, (int)e2, (int)e3};
    auto it = ctx->modup_range_tables.find(key);
    if (it != ctx->modup_range_tables.end()) return it->second;
    u32 lo = j * ctx->alpha, hi = std::min((j + 1) * ctx->alpha, level + 1);
    std::vector<u32> in, out;
    for (u32 i = lo; i < hi; i++) in.push_back(i);
    for (u32 e = e0; e < e1; e++) out.push_back(ctx->ext_mod(e, level));
    for (u32 e = e2; e < e3; e++) out.push_back(ctx->ext_mod(e, level));
    return ctx->modup_range_tables[key] = build_table(ctx, in, out);
}

const ConvTable& moddown_table(vr_context* ctx, u32 level)
{
    std::lock_guard<std::mutex> g(ctx->mu);
    auto it = ctx->moddown_tables.find((int)level);
    if (it != ctx->moddown_tables.end()) return it->second;
    std::vector<u32> in, out;
    for (u32 k = 0; k < ctx->K; k++) in.push_back(ctx->L + 1 + k);
    for (u32 i = 0; i <= level; i++) out.push_back(i);
    return ctx->moddown_tables[(int)level] = build_table(ctx, in, out);
}

// {q_l, p_0, ..., p_{K-1}} -> q_0..q_{nk-1} (nk <= l): the conversion of a
// ModDown that also drops q_l (relinearisation fused with the rescale), to
// the nk limbs the consumer reads
const ConvTable& moddown_rs_table(vr_context* ctx, u32 level, u32 nk)
{
    std::lock_guard<std::mutex> g(ctx->mu);
    const int key = (int)(level * 1024 + nk);
    auto it = ctx->moddown_rs_tables.find(key);
    if (it != ctx->moddown_rs_tables.end()) return it->second;
    std::vector<u32> in{level}, out;
    for (u32 k = 0; k < ctx->K; k++) in.push_back(ctx->L + 1 + k);
    for (u32 i = 0; i < nk; i++) out.push_back(i);
    return ctx->moddown_rs_tables[key] = build_table(ctx, in, out);
}

void launch_alu(vr_context* ctx, const ConvArgs& a, u32 n_polys, hipStream_t s)
{
    dim3 grid((ctx->n + kThreads - 1) / kThreads, n_polys);
    hipLaunchKernelGGL(k_base_convert, grid, dim3(kThreads), 0, s, a);
    VR_CHECK_LAUNCH();
}

void launch_mfma(vr_context* ctx, const ConvArgs& a, const ConvTable& tb, u32 n_polys, hipStream_t s)
{
    static std::once_flag attr;
    std::call_once(attr, [] {
        (void)hipFuncSetAttribute((const void*)k_base_convert_mfma,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    });
    const size_t shmem = ((size_t)tb.groups * 4 * tb.steps * 64 + (size_t)4 * tb.steps * kDigitRow) * 8;
    // a few polynomials per block so the constant table is staged into LDS
    // about 4k times per call, not once per 256 coefficients of every poly
    const u32 xblocks = ctx->n / kMfmaCoef;
    const u32 ypolys = std::max(1u, std::min(n_polys, (4096 + xblocks - 1) / xblocks));
    hipLaunchKernelGGL(k_base_convert_mfma, dim3(xblocks, ypolys), dim3(256), shmem, s, a, tb.wt,
                       tb.steps, tb.groups, n_polys);
    VR_CHECK_LAUNCH();
}

// The FP64 kernel takes at most one input of 2^51 or more, and only as the
// first (q_0 in digit 0); other tables stay on the integer kernels.
bool fp_usable(const ConvTable& tb) { return tb.wf && (tb.wide & ~1u) == 0; }

template <bool W0>
void launch_fp_w(const ConvArgs& a, const ConvFp& f, dim3 grid, hipStream_t s)
{
    if (a.n_in <= 4)
        hipLaunchKernelGGL((k_base_convert_fp<4, W0>), grid, dim3(kThreads), 0, s, a, f);
    else if (a.n_in <= 8)
        hipLaunchKernelGGL((k_base_convert_fp<8, W0>), grid, dim3(kThreads), 0, s, a, f);
    else if (a.n_in == 9)   // digits of nine primes
        hipLaunchKernelGGL((k_base_convert_fp<9, W0>), grid, dim3(kThreads), 0, s, a, f);
    else if (a.n_in == 10)  // nine special primes and q_l (ModDown with the rescale)
        hipLaunchKernelGGL((k_base_convert_fp<10, W0>), grid, dim3(kThreads), 0, s, a, f);
    else if (a.n_in <= 12)
        hipLaunchKernelGGL((k_base_convert_fp<12, W0>), grid, dim3(kThreads), 0, s, a, f);
    else
        hipLaunchKernelGGL((k_base_convert_fp<16, W0>), grid, dim3(kThreads), 0, s, a, f);
}

void launch_fp(vr_context* ctx, const ConvArgs& a, const ConvTable& tb, u32 n_polys, hipStream_t s)
{
    ConvFp f;
    f.w = tb.wf;
    f.t = tb.wf + (size_t)tb.n_out * kMaxIn * 2;
    dim3 grid((ctx->n + kThreads - 1) / kThreads, n_polys);
    if (tb.wide & 1)
        launch_fp_w<true>(a, f, grid, s);
    else
        launch_fp_w<false>(a, f, grid, s);
    VR_CHECK_LAUNCH();
}

bool mfma_usable(vr_context* ctx, const ConvTable& tb)
{
    const size_t shmem = ((size_t)tb.groups * 4 * tb.steps * 64 + (size_t)4 * tb.steps * kDigitRow) * 8;
    return ctx->n >= kMfmaCoef && tb.wt && shmem <= 160 * 1024;
}

// The kernels give the same words, so the first call of a table runs each
// once on the real operands under events and keeps the fastest.
void launch_convert(vr_context* ctx, const ConvArgs& a, const ConvTable& tb, u32 n_polys,
                    hipStream_t s)
{
    ProfScope prof(ctx, kProfBaseConv, s, (u64)n_polys * a.n_out);
    int mode = 0;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->tuning.find("base_convert");
        if (it != ctx->tuning.end()) mode = it->second;
    }
    const bool mfma = mfma_usable(ctx, tb), fp = fp_usable(tb);
    // split: only target 0 is 2^51 or more (q_0 first among narrow targets)
    const bool split = fp && tb.n_out >= 2 && tb.wide_out == 1u;
    auto launch_split = [&]() {
        ConvArgs b = a;
        b.o_lo = 1;
        launch_fp(ctx, b, tb, n_polys, s);
        ConvArgs w = a;
        w.o_lo = 0;
        w.o_hi = 1;
        launch_alu(ctx, w, n_polys, s);
    };
    if (mode == 1 || (mode == 2 && !mfma) || (mode == 3 && !fp)) return launch_alu(ctx, a, n_polys, s);
    if (mode == 2) return launch_mfma(ctx, a, tb, n_polys, s);
    if (mode == 3) return launch_fp(ctx, a, tb, n_polys, s);
    if (mode == 4) return split ? launch_split() : fp ? launch_fp(ctx, a, tb, n_polys, s) : launch_alu(ctx, a, n_polys, s);
    int c = tb.choice->load();
    if (c < 0 && !g_capture && ctx->prof.cls < 0) {
        // every candidate twice (each writes the same words; the first
        // launch of a kernel also pays for loading it), the faster of each
        // candidate's two runs counts.  split is not a candidate: it never
        // won a clean comparison, and a first call timed while other
        // streams run (the server's waves) could pick it by noise.
        hipEvent_t ev[4];
        for (auto& e : ev) VR_HIP(hipEventCreate(&e));
        float ms[3] = {1e30f, 1e30f, 1e30f};
        for (int round = 0; round < 2; round++) {
            VR_HIP(hipEventRecord(ev[0], s));
            launch_alu(ctx, a, n_polys, s);
            VR_HIP(hipEventRecord(ev[1], s));
            if (fp) launch_fp(ctx, a, tb, n_polys, s);
            VR_HIP(hipEventRecord(ev[2], s));
            if (mfma) launch_mfma(ctx, a, tb, n_polys, s);
            VR_HIP(hipEventRecord(ev[3], s));
            VR_HIP(hipEventSynchronize(ev[3]));
            for (int k = 0; k < 3; k++) {
                float t = 0;
                VR_HIP(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
                ms[k] = std::min(ms[k], t);
            }
        }
        for (auto& e : ev) (void)hipEventDestroy(e);
        // choice codes: 0 alu (ms[0]), 2 fp64 (ms[1]), 1 mfma (ms[2])
        int pick = 0;
        float best = ms[0];
        if (fp && ms[1] < best) pick = 2, best = ms[1];
        if (mfma && ms[2] < best) pick = 1, best = ms[2];
        tb.choice->store(pick);
        return;
    }
    if (c == 1) return launch_mfma(ctx, a, tb, n_polys, s);
    if (c == 2) return launch_fp(ctx, a, tb, n_polys, s);
    if (c == 3) return launch_split();
    launch_alu(ctx, a, n_polys, s);
}

}  // namespace

KsShape ks_shape(vr_context* ctx, u32 level)
{
    KsShape k;
    k.level = level;
    k.nq = level + 1;
    k.next = level + 1 + ctx->K;
    k.beta = (level + 1 + ctx->alpha - 1) / ctx->alpha;
    return k;
}

size_t keyswitch_modup_scratch(vr_context* ctx, u32 level)
{
    KsShape k = ks_shape(ctx, level);
    return ((size_t)k.beta * k.next + k.nq) * ctx->n;
}

size_t keyswitch_moddown_scratch(vr_context* ctx, u32 level, u32 n_ct)
{
    KsShape k = ks_shape(ctx, level);
    return (size_t)n_ct * 2 * (ctx->K + k.nq) * ctx->n;
}

// d_c = d + c * d_stride: [nq][N] evaluation domain, c < n_ct.
// X_c = X + c * beta * next * N: [beta][next][N].  coef: [n_ct][nq][N] scratch.
void keyswitch_modup_batch(vr_context* ctx, const u64* d, u64 d_stride, u32 n_ct, u32 level,
                           u64* X, u64* coef, hipStream_t s, u32 keep_q)
{
    KsShape k = ks_shape(ctx, level);
    const u32 n = ctx->n;
    const u64 xs = (u64)k.beta * k.next * n;
    // coefficient form of every d_c
    LimbSet ls = poly_limbs(const_cast<u64*>(d), coef, n_ct, k.nq, d_stride, (int)level);
    ls.out_dense = 1;
    ntt_inverse(ctx, ls, s);
    if (keep_q && ctx->alpha > 1) {
        // only the extended limbs the inner product will read, q_0..q_{keep-1},
        // q_level and the special primes, outside each digit's own limbs: per
        // digit at most three runs, each transformed on its own.  Two runs
        // share one conversion (the gap between them is the kernels' output
        // skip), so the digit's inputs are read and centred once; three
        // convert one by one.
        if (keep_q > level) throw Error(VR_EINVAL, "ModUp: kept limbs above the level");
        for (u32 j = 0; j < k.beta; j++) {
            const u32 lo = j * ctx->alpha, hi = std::min((j + 1) * ctx->alpha, k.nq);
            std::vector<std::pair<u32, u32>> runs;
            if (std::min(keep_q, lo) > 0) runs.push_back({0, std::min(keep_q, lo)});
            if (hi < keep_q) runs.push_back({hi, keep_q});
            runs.push_back({std::max(level, hi), k.next});
            auto convert = [&](u32 e0, u32 e1, u32 e2, u32 e3) {
                const ConvTable& tb = modup_range_table(ctx, level, j, e0, e1, e2, e3);
                ConvArgs a;
                a.in = coef + (size_t)lo * n;
                a.in_stride = (u64)k.nq * n;
                a.out = X + ((size_t)j * k.next + e0) * n;
                a.out_stride = xs;
                a.skip_at = e3 > e2 ? e1 - e0 : 0xffffffffu;
                a.skip_len = e3 > e2 ? e2 - e1 : 0;
                a.tab = tb.dev;
                a.n_in = tb.n_in;
                a.n_out = tb.n_out;
                a.log_n = ctx->log_n;
                a.mq = ctx->d_modq;
                launch_convert(ctx, a, tb, n_ct, s);
            };
            if (runs.size() == 2)
                convert(runs[0].first, runs[0].second, runs[1].first, runs[1].second);
            for (const auto& r : runs) {
                if (runs.size() != 2) convert(r.first, r.second, 0, 0);
                LimbSet t = poly_limbs(X + (size_t)j * k.next * n, X + (size_t)j * k.next * n, n_ct,
                                       r.second - r.first, xs, (int)level);
                t.slot0 = r.first;
                ntt_forward(ctx, t, s);
            }
        }
        return;
    }
    // one-limb digits: the conversion is a centred reduction, done by the
    // NTT as it loads each limb (below); wider digits convert first
    const bool fused = ctx->alpha == 1;
    for (u32 j = 0; j < k.beta; j++) {
        u32 lo = j * ctx->alpha, hi = std::min((j + 1) * ctx->alpha, k.nq);
        if (!fused) {
            const ConvTable& tb = modup_table(ctx, level, j);
            ConvArgs a;
            a.in = coef + (size_t)lo * n;
            a.in_stride = (u64)k.nq * n;
            a.out = X + (size_t)j * k.next * n;
            a.out_stride = xs;
            a.skip_at = lo;
            a.skip_len = hi - lo;
            a.tab = tb.dev;
            a.n_in = tb.n_in;
            a.n_out = tb.n_out;
            a.log_n = ctx->log_n;
            a.mq = ctx->d_modq;
            launch_convert(ctx, a, tb, n_ct, s);
        }
    }
    // each digit's own limbs are d itself (already in the evaluation domain):
    // the inner product reads them there, so they are not copied into X
    // every converted limb of every digit to the evaluation domain: per digit
    // all limbs except the digit's own (digit_skip), the uniform count being
    // next - alpha; a short last digit leaves alpha - last more limbs.
    LimbSet t = poly_limbs(X, X, n_ct * k.beta, k.next - ctx->alpha, (u64)k.next * n, (int)level);
    t.digit_skip = 1;
    t.alpha = ctx->alpha;
    t.beta = k.beta;
    t.nq = k.nq;
    if (fused) {
        t.cv_src = coef;             // digit j of ciphertext c: coef + c * nq * N + j * N
        t.cv_ct_stride = (u64)k.nq * n;
        t.cv_beta = k.beta;
        t.cv_mod0 = 0;
    }
    ntt_forward(ctx, t, s);
    u32 last = k.nq - (k.beta - 1) * ctx->alpha;
    if (last < ctx->alpha) {
        LimbSet r = poly_limbs(X + (size_t)(k.beta - 1) * k.next * n, nullptr, n_ct,
                               ctx->alpha - last, xs, (int)level);
        r.out = r.in;
        r.slot0 = k.next - ctx->alpha + last;
        ntt_forward(ctx, r, s);
    }
}

void keyswitch_modup(vr_context* ctx, const u64* d, u32 level, u64* X, u64* coef, hipStream_t s)
{
    keyswitch_modup_batch(ctx, d, (u64)(level + 1) * ctx->n, 1, level, X, coef, s);
}

namespace {

// inverse of g modulo 2N: the odd residues mod 2N = 2^(log N + 1) have
// exponent N/2, so g^-1 = g^(N/2 - 1)
u32 galois_inverse(vr_context* ctx, u32 g)
{
    const u64 two_n = 2ull * ctx->n;
    if (g == 1) return 1;
    u64 r = 1;
    for (u64 x = g % two_n, ee = two_n / 4 - 1; ee; ee >>= 1, x = x * x % two_n)
        if (ee & 1) r = r * x % two_n;
    if (r * g % two_n != 1) throw Error(VR_EINVAL, "key switching: no inverse Galois element");
    return (u32)r;
}

void ks_inner_launch(vr_context* ctx, const u64* X, u64 x_stride, const u64* d, u64 d_stride, u32 n_ct,
                     const KsSteps& st, u32 ns, u32 level, u64 u_stride, hipStream_t s, const u64* fold_c0,
                     u64 fold_stride, u32 keep_q)
{
    KsShape k = ks_shape(ctx, level);
    // at least ~4096 blocks: split the ciphertexts (each group re-reads the key)
    u32 bxy = ((ctx->n + kThreads - 1) / kThreads) * k.next;
    u32 groups = (4096 + bxy - 1) / bxy;
    if (groups > n_ct) groups = n_ct;
    if (groups < 1) groups = 1;
    dim3 grid((ctx->n + kThreads - 1) / kThreads, k.next, groups);
    const u32 u_limbs = keep_q ? keep_q + 1 + ctx->K : k.next;
    if (keep_q > level) throw Error(VR_EINVAL, "key switching: kept limbs above the level");
    ProfScope prof(ctx, kProfKsInner, s, (u64)n_ct * u_limbs * ns);
    if (k.beta > 16) throw Error(VR_EINVAL, "key switching: more than 16 digits");
    // one launch per path (FP64 below 2^51, else integer) over its runs of
    // consecutive extended limbs, so each kernel gets its own registers
    for (int pass = 0; pass < 2; pass++) {
        const bool fp = pass == 0;
        std::vector<std::pair<u32, u32>> runs;   // (begin, length)
        for (u32 e = 0; e < k.next; e++) {
            if ((ctx->modq[ctx->ext_mod(e, level)].q < (1ull << 51)) != fp) continue;
            if (keep_q && e >= keep_q && e < level) continue;   // Q limbs nobody reads
            if (!runs.empty() && runs.back().first + runs.back().second == e)
                runs.back().second++;
            else
                runs.push_back({e, 1});
        }
        for (size_t r0 = 0; r0 < runs.size(); r0 += kMaxRuns) {
            LimbRuns lr = {};
            u32 rows = 0;
            for (size_t r = r0; r < std::min(runs.size(), r0 + kMaxRuns); r++) {
                const u32 b = runs[r].first;
                lr.b[r - r0] = b;
                lr.len[r - r0] = runs[r].second;
                lr.o[r - r0] = keep_q && b >= level ? b - level + keep_q : b;
                rows += runs[r].second;
            }
            dim3 g2(grid.x, rows, grid.z);
#define VR_KS_INNER(B, F, S)                                                                               \
    hipLaunchKernelGGL((k_ks_inner<B, F, S>), g2, dim3(kThreads), 0, s, X, x_stride, d, d_stride, n_ct, st,   \
                       ctx->nmod(), level, k.next, k.beta, ctx->alpha, ctx->L, ctx->log_n, u_stride, ctx->d_modq, \
                       lr, fold_c0, fold_stride, ctx->d_pmod_tab, u_limbs)
#define VR_KS_INNER_S(B, F)      \
    if (ns == 2)                 \
        VR_KS_INNER(B, F, 2);    \
    else                         \
        VR_KS_INNER(B, F, 1)
            if (k.beta <= 4) {
                if (fp)
                    VR_KS_INNER_S(4, true);
                else
                    VR_KS_INNER_S(4, false);
            } else if (k.beta <= 8) {
                if (fp)
                    VR_KS_INNER_S(8, true);
                else
                    VR_KS_INNER_S(8, false);
            } else {
                if (fp)
                    VR_KS_INNER(16, true, 1);
                else
                    VR_KS_INNER(16, false, 1);
            }
#undef VR_KS_INNER_S
#undef VR_KS_INNER
            VR_CHECK_LAUNCH();
        }
    }
}

}  // namespace

void keyswitch_inner_batch(vr_context* ctx, const u64* X, u64 x_stride, const u64* d, u64 d_stride,
                           u32 n_ct, const u64* key, u32 level, u32 g, u64* U, u64 u_stride,
                           hipStream_t s, const u64* fold_c0, u64 fold_stride, u32 keep_q)
{
    KsSteps st = {};
    st.key[0] = key;
    st.U[0] = U;
    st.g_inv[0] = galois_inverse(ctx, g);
    ks_inner_launch(ctx, X, x_stride, d, d_stride, n_ct, st, 1, level, u_stride, s, fold_c0, fold_stride, keep_q);
}

void keyswitch_inner_batch2(vr_context* ctx, const u64* X, u64 x_stride, const u64* d, u64 d_stride,
                            u32 n_ct, const u64* key0, const u64* key1, u32 level, u32 g0, u32 g1, u64* U0,
                            u64* U1, u64 u_stride, hipStream_t s, const u64* fold_c0, u64 fold_stride,
                            u32 keep_q)
{
    if (ks_shape(ctx, level).beta > 8) {   // one step at a time (registers)
        keyswitch_inner_batch(ctx, X, x_stride, d, d_stride, n_ct, key0, level, g0, U0, u_stride, s, fold_c0,
                              fold_stride, keep_q);
        keyswitch_inner_batch(ctx, X, x_stride, d, d_stride, n_ct, key1, level, g1, U1, u_stride, s, fold_c0,
                              fold_stride, keep_q);
        return;
    }
    KsSteps st = {};
    st.key[0] = key0;
    st.key[1] = key1;
    st.U[0] = U0;
    st.U[1] = U1;
    st.g_inv[0] = galois_inverse(ctx, g0);
    st.g_inv[1] = galois_inverse(ctx, g1);
    ks_inner_launch(ctx, X, x_stride, d, d_stride, n_ct, st, 2, level, u_stride, s, fold_c0, fold_stride, keep_q);
}


void keyswitch_inner(vr_context* ctx, const u64* X, const u64* d, const u64* key, u32 level, u32 g,
                     u64* U, hipStream_t s)
{
    KsShape k = ks_shape(ctx, level);
    keyswitch_inner_batch(ctx, X, (u64)k.beta * k.next * ctx->n, d, (u64)k.nq * ctx->n, 1, key, level, g,
                          U, (u64)2 * k.next * ctx->n, s);
}

void keyswitch_moddown_batch(vr_context* ctx, u64* U, u64 u_stride, u32 n_ct, u32 level,
                             u64* out0, u64* out1, u64 out_stride, const u64* add0, u32 add0_g,
                             const u64* add1, u64 add_stride, u64* scratch, hipStream_t s)
{
    KsShape k = ks_shape(ctx, level);
    const u32 n = ctx->n, K = ctx->K;
    if (u_stride != (u64)2 * k.next * n) throw Error(VR_EINVAL, "moddown: U blocks must be dense");
    u64* pcoef = scratch;                                   // [n_ct*2][K][N]
    u64* Y = scratch + (size_t)n_ct * 2 * K * n;            // [n_ct*2][nq][N]
    // special-prime limbs to the coefficient domain
    LimbSet ls = poly_limbs(U, pcoef, n_ct * 2, K, (u64)k.next * n, (int)level);
    ls.slot0 = k.nq;
    ls.out_dense = 1;
    ntt_inverse(ctx, ls, s);
    LimbSet ly = poly_limbs(Y, Y, n_ct * 2, k.nq, (u64)k.nq * n, (int)level);
    if (K == 1) {
        // one special prime: the conversion is a centred reduction done by the
        // NTT as it loads each limb
        ly.cv_src = pcoef;
        ly.cv_ct_stride = n;
        ly.cv_beta = 1;
        ly.cv_mod0 = ctx->L + 1;
    } else {
        const ConvTable& tb = moddown_table(ctx, level);
        ConvArgs a;
        a.in = pcoef;
        a.in_stride = (u64)K * n;
        a.out = Y;
        a.out_stride = (u64)k.nq * n;
        a.skip_at = 0xffffffffu;
        a.skip_len = 0;
        a.tab = tb.dev;
        a.n_in = tb.n_in;
        a.n_out = tb.n_out;
        a.log_n = ctx->log_n;
        a.mq = ctx->d_modq;
        launch_convert(ctx, a, tb, n_ct * 2, s);
    }
    // (U - Y) P^-1 (+ add) in the forward transform's last round where the
    // plan allows, else by the finish kernel
    NttEpilogue& ep = ly.epi;
    ep.a = U;
    ep.a_ct = u_stride;
    ep.a_comp = (u64)k.next * n;
    ep.out0 = out0;
    ep.out1 = out1;
    ep.out_ct = out_stride;
    ep.add0 = add0;
    ep.add1 = add1;
    ep.add_ct = add_stride;
    ep.add0_g = add0_g;
    ep.cmul = ctx->d_pinv_tab;
    if (ntt_forward(ctx, ly, s)) return;
    dim3 grid((n + kThreads - 1) / kThreads, n_ct * k.nq);
    ProfScope prof(ctx, kProfModDown, s, (u64)n_ct * 2 * k.nq);
    hipLaunchKernelGGL(k_moddown_finish, grid, dim3(kThreads), 0, s, U, u_stride, Y, k.nq, k.next,
                       ctx->log_n, out0, out1, out_stride, add0, add0_g, add1, add_stride,
                       ctx->d_modq, ctx->d_pinv_tab, (const ulonglong2*)nullptr);
    VR_CHECK_LAUNCH();
}

// Relinearisation and rescale as one ModDown by P q_l (l = level): v_j = U_j
// + P c_j on the Q limbs (U_j on the special ones, where P c_j vanishes), and
//   out_j,i = (v_j,i - conv(v_j over {q_l, P})_i) (P q_l)^-1
//           = (U_j,i - y_j,i) (P q_l)^-1 + c_j,i q_l^-1,   i < l,
// so only the q_l limb takes the fold of P c_j before the conversion.  With
// c0 = c1 = null, U is already the whole extended ciphertext v.  keep_q = nk
// > 0: U is compact ([2][nk + 1 + K][N]: q_0..q_{nk-1}, q_l, the special
// primes) and only output limbs 0..nk-1 are made (level nk - 1).
void keyswitch_moddown_rescale_batch(vr_context* ctx, u64* U, u64 u_stride, u32 n_ct, u32 level,
                                     u64* out0, u64* out1, u64 out_stride, const u64* c0,
                                     const u64* c1, u64 c_stride, u64* scratch, hipStream_t s, u32 keep_q)
{
    if (level == 0) throw Error(VR_ELEVEL, "no limb left to rescale by");
    if (keep_q > level) throw Error(VR_EINVAL, "moddown-rescale: kept limbs above the level");
    const u32 n = ctx->n, K = ctx->K, nd = K + 1, no = keep_q ? keep_q : level;
    const u32 ul = no + 1 + K;   // limbs of U per component; q_l at limb no
    if (u_stride != (u64)2 * ul * n) throw Error(VR_EINVAL, "moddown: U blocks must be dense");
    if (!c0 != !c1) throw Error(VR_EINVAL, "moddown-rescale: c0 and c1 come together");
    u64* dcoef = scratch;                                   // [n_ct*2][K+1][N]
    u64* Y = scratch + (size_t)n_ct * 2 * nd * n;           // [n_ct*2][no][N]
    if (c0) {
        const u64 ql = ctx->mod[level];
        u64 pm = 1 % ql;
        for (u32 j = 0; j < K; j++) pm = (u64)((u128)pm * (ctx->mod[ctx->L + 1 + j] % ql) % ql);
        dim3 grid((n + kThreads - 1) / kThreads, n_ct * 2);
        hipLaunchKernelGGL(k_fold_pc, grid, dim3(kThreads), 0, s, U + (size_t)no * n, u_stride,
                           (u64)ul * n, c0 + (size_t)level * n, c1 + (size_t)level * n, c_stride, pm,
                           shoup_companion(pm, ql), ql, n);
        VR_CHECK_LAUNCH();
    }
    // q_l and the special limbs (consecutive in U) to the coefficient domain
    LimbSet ls = poly_limbs(U, dcoef, n_ct * 2, nd, (u64)ul * n, (int)no);
    ls.slot0 = no;
    ls.out_dense = 1;
    ls.remap_slot = no;
    ls.remap_mod = level;
    ntt_inverse(ctx, ls, s);
    const ConvTable& tb = moddown_rs_table(ctx, level, no);
    ConvArgs a;
    a.in = dcoef;
    a.in_stride = (u64)nd * n;
    a.out = Y;
    a.out_stride = (u64)no * n;
    a.skip_at = 0xffffffffu;
    a.skip_len = 0;
    a.tab = tb.dev;
    a.n_in = tb.n_in;
    a.n_out = tb.n_out;
    a.log_n = ctx->log_n;
    a.mq = ctx->d_modq;
    launch_convert(ctx, a, tb, n_ct * 2, s);
    LimbSet ly = poly_limbs(Y, Y, n_ct * 2, no, (u64)no * n, (int)level);
    NttEpilogue& ep = ly.epi;
    ep.a = U;
    ep.a_ct = u_stride;
    ep.a_comp = (u64)ul * n;
    ep.out0 = out0;
    ep.out1 = out1;
    ep.out_ct = out_stride;
    ep.add0 = c0;
    ep.add1 = c1;
    ep.add_ct = c_stride;
    ep.cmul = ctx->d_prinv_tab + (size_t)level * ctx->nmod();
    ep.bmul = c0 ? ctx->d_rinv_tab + (size_t)level * ctx->nmod() : nullptr;
    if (ntt_forward(ctx, ly, s)) return;
    dim3 grid((n + kThreads - 1) / kThreads, n_ct * no);
    ProfScope prof(ctx, kProfModDown, s, (u64)n_ct * 2 * no);
    hipLaunchKernelGGL(k_moddown_finish, grid, dim3(kThreads), 0, s, U, u_stride, Y, no, ul,
                       ctx->log_n, out0, out1, out_stride, c0, 1u, c1, c_stride, ctx->d_modq,
                       ctx->d_prinv_tab + (size_t)level * ctx->nmod(),
                       ctx->d_rinv_tab + (size_t)level * ctx->nmod());
    VR_CHECK_LAUNCH();
}

void keyswitch_moddown(vr_context* ctx, u64* U, u32 level, u64* out0, u64* out1, const u64* add0,
                       u32 add0_g, const u64* add1, u64* scratch, hipStream_t s)
{
    KsShape k = ks_shape(ctx, level);
    keyswitch_moddown_batch(ctx, U, (u64)2 * k.next * ctx->n, 1, level, out0, out1, 0, add0,
                            add0_g, add1, 0, scratch, s);
}

}  // namespace vr
