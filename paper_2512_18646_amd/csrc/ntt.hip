// Negacyclic NTT / inverse NTT on gfx950.
//
// Transform: out[i] = sum_t a_t psi^((2 brev(i) + 1) t) mod q (bit-reversed
// evaluation order), the radix-2 Cooley-Tukey network with merged psi
// twiddles; the inverse is the Gentleman-Sande network with inverse twiddles
// followed by N^-1.
//
// Layout.  A limb is N uint64 (64 KiB at N = 2^13, 128 KiB at 2^14, 512 KiB at
// 2^16).  Up to 2^14 one workgroup holds a whole limb in LDS (160 KiB per CU)
// and runs every stage there: one HBM read and one write per limb.  At 2^15
// and 2^16 the stages split in two passes over groups of 2^7-2^8 elements; the
// first pass works on strided groups with 16-32 consecutive groups per
// workgroup so each row read is a coalesced 128-256 byte segment, the second
// on contiguous blocks.
//
// Compute.  Inside a pass the stages run in rounds of up to four: each thread
// pulls a 16-element group (elements that differ only in the four index bits
// those stages touch) from LDS into registers, issues the 15 twiddle loads of
// the round at once (16-byte (w, w') pairs, w' = floor(w 2^64 / q)), runs the
// 32 butterflies, and writes the group back: one LDS round trip and one
// barrier per four stages.  LDS rows are padded by one word every 16 so the
// stride-16 group reads of the last round do not collide on banks.  Shoup
// products with lazy reduction keep forward values in [0, 4q) and inverse
// values in [0, 2q) (Harvey 2014); the last pass stores [0, q).
//
// Moduli below 2^51 take an FP64 path instead (one branch per workgroup, as
// a workgroup holds one limb): values are integers held exactly in doubles in
// balanced form, a product y w mod q is p = y w, e = fma(y, w, -p) (the exact
// low part), t = rint(p / q), r = fma(-t, q, p) + e -- six FP64 operations,
// all exact while |values| < 2^53 -- and the butterflies add and subtract
// without any correction.  Bounds: from |x| <= q/2, a product is off the
// nearest multiple by at most q/2 plus the rounding of p / q (< 0.7 q while
// |p| < 1.4 q^2) plus |e| (< q/4), so each forward stage adds < 1.44 q; four
// stages stay below 6.2 q < 2^52.7 for q < 2^50, two stages below 3.4 q for
// q < 2^51, and two inverse stages (whose sums double) below 2.9 q.  A
// balanced reduction x - q rint(x / q) follows every such group of stages.
// Between the passes of a two-pass transform the balanced doubles themselves
// go through memory; the last pass stores the canonical uint64.
#include "vr_core.h"

namespace vr {

struct NttPass {
    LimbSet ls;
    const ModQ* mq;
    const u64* tw;      // [nmod][N][2]
    const double* twf;  // [nmod][N] balanced
    u32 log_n, L;
    u32 s0, log_g, log_c;
    u32 first, last;
    u32 max_r;          // stages per round (4, or 5 with 32 elements per thread)
    u32 r0;             // first limb of this launch (launches over chunks of limbs)
};
VR_KERNEL_ARG(NttPass);

__device__ __forceinline__ void limb_addr(const LimbSet& ls, u32 r, u32 n, u32 L,
                                          const u64** in, u64** out, u32* mod)
{
    u32 poly = r / ls.per_poly;
    u32 l = r - poly * ls.per_poly;
    u32 skip_at = ls.skip_at, skip_len = ls.skip_len;
    if (ls.digit_skip) {
        u32 d = poly % ls.beta;
        skip_at = d * ls.alpha;
        u32 end = skip_at + ls.alpha;
        skip_len = (end > ls.nq ? ls.nq : end) - skip_at;
    }
    u32 slot = ls.slot0 + (l < skip_at ? l : l + skip_len);
    *mod = ((int)slot <= ls.level) ? slot : (u32)((int)L + 1 + (int)slot - ls.level - 1);
    if (slot == ls.remap_slot) *mod = ls.remap_mod;
    size_t off = (size_t)poly * ls.poly_stride + (size_t)slot * n;
    *in = ls.in + off;
    *out = ls.out_dense ? ls.out + (size_t)r * n : ls.out + off;
}

// Dispatch order of a set's limbs: slot l of every poly before slot l + 1,
// so limbs that share a modulus, and so its twiddle tables, run close
// together and the tables are read from each XCD's L2 rather than from HBM
// once per limb.  rr (dispatch index) -> r = poly * per_poly + l.
__device__ __forceinline__ u32 limb_order(const LimbSet& ls, u32 rr)
{
    const u32 np = ls.n_polys;
    if (np <= 1) return rr;
    const u32 l = rr / np;
    return (rr - l * np) * ls.per_poly + l;
}

__device__ __forceinline__ u32 pad(u32 i) { return i + (i >> 4); }

// words per thread moved between global memory and LDS with their loads all
// issued before the first is used
constexpr int kBatch = 16;

// Where a round reads and writes.  A pass that holds the whole limb takes its
// first round straight from global memory (element e at gsrc[e]: the groups
// of the first forward round are strided so consecutive threads read
// consecutive words) and writes its last round straight back in final form,
// saving two LDS round trips and letting each wave start and finish on its
// own instead of at a barrier.
struct RoundIO {
    const u64* gsrc = nullptr;   // canonical uint64 input
    u64* gdst = nullptr;         // canonical uint64 output
    u64 cq = 0;                  // != 0: gsrc holds residues mod cq, converted on the load
    u64 t_one_s = 0;             // floor(2^64 / q) of the limb's own modulus
};

// centred residue v mod cq as a residue mod q (one-limb fast base conversion)
__device__ __forceinline__ u64 conv_one(u64 v, u64 cq, u64 q, u64 one_s)
{
    const bool neg = v > (cq >> 1);
    u64 x = neg ? cq - v : v;
    x = csub(shoup_lazy(x, 1, one_s, q), q);
    return neg ? neg_mod(x, q) : x;
}

// Whether every lane of a wave has the same twiddle prefix in a round: the
// group's block index H is common when the strided groups of a workgroup do
// not cross a row (lo_bits >= log_c) or a wave stays in one group column
// (log_g - R >= 6), and the in-group prefix hi is common when a wave's 64
// lanes differ only below it (low_bits >= 6) or it is empty (sg0 = 0).
// Then the twiddles are loaded once per wave through the scalar cache.
__device__ __forceinline__ bool wave_uniform_prefix(u32 lo_bits, u32 log_c, u32 log_g, u32 R,
                                                    u32 low_bits, u32 sg0)
{
    return (lo_bits >= log_c || log_g - R >= 6) && (low_bits >= 6 || sg0 == 0);
}

template <int R, bool INV, bool UNI>
__device__ __forceinline__ void int_butterflies(u64 (&x)[1 << R], const ulonglong2* twp, u32 hprefix,
                                                u32 s_pass, u32 sg0, u64 q)
{
    if (UNI) hprefix = __builtin_amdgcn_readfirstlane(hprefix);
    const u64 q2 = 2 * q;
    if (!INV) {
#pragma unroll
        for (int k = 0; k < R; k++) {
            const int half = 1 << (R - 1 - k);
            const u32 tb = (1u << (s_pass + sg0 + k)) + (hprefix << k);
#pragma unroll
            for (int j = 0; j < (1 << k); j++) {
                const ulonglong2 t = twp[tb + j];
                const u64 wv = t.x, wsv = t.y;
#pragma unroll
                for (int i = 0; i < half; i++) {
                    const int m1 = (j << (R - k)) + i, m2 = m1 + half;
                    u64 X = x[m1];
                    X = X >= q2 ? X - q2 : X;
                    u64 T = shoup_lazy(x[m2], wv, wsv, q);
                    x[m1] = X + T;
                    x[m2] = X + q2 - T;
                }
            }
        }
    } else {
#pragma unroll
        for (int k = R - 1; k >= 0; k--) {
            const int half = 1 << (R - 1 - k);
            const u32 tb = (1u << (s_pass + sg0 + k)) + (hprefix << k);
#pragma unroll
            for (int j = 0; j < (1 << k); j++) {
                const ulonglong2 t = twp[tb + j];
                const u64 wv = t.x, wsv = t.y;
#pragma unroll
                for (int i = 0; i < half; i++) {
                    const int m1 = (j << (R - k)) + i, m2 = m1 + half;
                    u64 X = x[m1], Y = x[m2];
                    u64 S = X + Y;
                    x[m1] = S >= q2 ? S - q2 : S;
                    x[m2] = shoup_lazy(X + q2 - Y, wv, wsv, q);
                }
            }
        }
    }
}

// One round of R stages (local stages sg0 .. sg0+R-1 of the pass) over every
// 2^R-element group of the tile.
template <int R, bool INV, int THREADS>
__device__ __forceinline__ void ntt_round(u64* lds, const u64* tw, const ModQ& mq, u32 log_g,
                                          u32 log_c, u32 sg0, u32 s_pass, u32 g0, u32 lo_bits,
                                          RoundIO io)
{
    const u64 q = mq.q;
    constexpr int E = 1 << R;
    const u32 G = 1u << log_g;
    const u32 low_bits = log_g - sg0 - R;
    const u32 ngroups = (G >> R) << log_c;
    const u64 q2 = 2 * q;
    for (u32 f = threadIdx.x; f < ngroups; f += THREADS) {
        const u32 c = f >> (log_g - R);
        const u32 gid = f & ((G >> R) - 1);
        const u32 hi = gid >> low_bits;
        const u32 lo = gid & ((1u << low_bits) - 1);
        const u32 base = c * G + (hi << (log_g - sg0)) + lo;
        const u32 H = (g0 + c) >> lo_bits;
        const u32 hprefix = (H << sg0) | hi;
        // stage k of the round uses the 2^k consecutive twiddles starting at
        // 2^(s_pass + sg0 + k) + (hprefix << k)
        const ulonglong2* twp = (const ulonglong2*)tw;
        const bool uni = wave_uniform_prefix(lo_bits, log_c, log_g, R, low_bits, sg0);
        u64 x[E];
        if (io.gsrc) {
#pragma unroll
            for (int m = 0; m < E; m++) {
                x[m] = io.gsrc[base + ((u32)m << low_bits)];
                if (io.cq) x[m] = conv_one(x[m], io.cq, q, io.t_one_s);
            }
        } else {
#pragma unroll
            for (int m = 0; m < E; m++) x[m] = lds[pad(base + ((u32)m << low_bits))];
        }
        if (uni)
            int_butterflies<R, INV, true>(x, twp, hprefix, s_pass, sg0, q);
        else
            int_butterflies<R, INV, false>(x, twp, hprefix, s_pass, sg0, q);
        if (io.gdst) {
#pragma unroll
            for (int m = 0; m < E; m++) {
                u64 v = x[m];
                if (!INV) {
                    v = v >= q2 ? v - q2 : v;
                    v = v >= q ? v - q : v;
                } else {
                    v = shoup(v, mq.ninv, mq.ninv_s, q);
                }
                io.gdst[base + ((u32)m << low_bits)] = v;
            }
        } else {
#pragma unroll
            for (int m = 0; m < E; m++) lds[pad(base + ((u32)m << low_bits))] = x[m];
        }
    }
}


template <int R, bool INV, bool UNI>
__device__ __forceinline__ void fp_butterflies(double (&x)[1 << R], const double* tw, u32 hprefix,
                                               u32 s_pass, u32 sg0, double q, double qinv, bool every2)
{
    constexpr int E = 1 << R;
    if (UNI) hprefix = __builtin_amdgcn_readfirstlane(hprefix);
    if (!INV) {
#pragma unroll
        for (int k = 0; k < R; k++) {
            const int half = 1 << (R - 1 - k);
            const u32 tb = (1u << (s_pass + sg0 + k)) + (hprefix << k);
#pragma unroll
            for (int j = 0; j < (1 << k); j++) {
                const double w = tw[tb + j];
#pragma unroll
                for (int i = 0; i < half; i++) {
                    const int m1 = (j << (R - k)) + i, m2 = m1 + half;
                    const double X = x[m1];
                    const double T = fmulmod(x[m2], w, q, qinv);
                    x[m1] = X + T;
                    x[m2] = X - T;
                }
            }
            if (every2 && (k & 1) && k != R - 1) {
#pragma unroll
                for (int m = 0; m < E; m++) x[m] = fbal(x[m], q, qinv);
            }
        }
    } else {
#pragma unroll
        for (int k = R - 1; k >= 0; k--) {
            const int half = 1 << (R - 1 - k);
            const u32 tb = (1u << (s_pass + sg0 + k)) + (hprefix << k);
#pragma unroll
            for (int j = 0; j < (1 << k); j++) {
                const double w = tw[tb + j];
#pragma unroll
                for (int i = 0; i < half; i++) {
                    const int m1 = (j << (R - k)) + i, m2 = m1 + half;
                    const double X = x[m1], Y = x[m2];
                    x[m1] = X + Y;
                    x[m2] = fmulmod(X - Y, w, q, qinv);
                }
            }
            if (((R - k) & 1) == 0 && k != 0) {
#pragma unroll
                for (int m = 0; m < E; m++) x[m] = fbal(x[m], q, qinv);
            }
        }
    }
}

template <int R, bool INV, int THREADS>
__device__ __forceinline__ void ntt_round_fp(double* lds, const double* tw, double q, double qinv,
                                             bool every2, u32 log_g, u32 log_c, u32 sg0,
                                             u32 s_pass, u32 g0, u32 lo_bits, RoundIO io,
                                             double ninv_f)
{
    const u64 qi = (u64)q;
    constexpr int E = 1 << R;
    const u32 G = 1u << log_g;
    const u32 low_bits = log_g - sg0 - R;
    const u32 ngroups = (G >> R) << log_c;
    for (u32 f = threadIdx.x; f < ngroups; f += THREADS) {
        const u32 c = f >> (log_g - R);
        const u32 gid = f & ((G >> R) - 1);
        const u32 hi = gid >> low_bits;
        const u32 lo = gid & ((1u << low_bits) - 1);
        const u32 base = c * G + (hi << (log_g - sg0)) + lo;
        const u32 H = (g0 + c) >> lo_bits;
        const u32 hprefix = (H << sg0) | hi;
        const bool uni = wave_uniform_prefix(lo_bits, log_c, log_g, R, low_bits, sg0);
        double x[E];
        if (io.gsrc) {
#pragma unroll
            for (int m = 0; m < E; m++) {
                u64 v = io.gsrc[base + ((u32)m << low_bits)];
                if (io.cq) v = conv_one(v, io.cq, qi, io.t_one_s);
                x[m] = to_bal(v, qi, q);
            }
        } else {
#pragma unroll
            for (int m = 0; m < E; m++) x[m] = lds[pad(base + ((u32)m << low_bits))];
        }
        if (uni)
            fp_butterflies<R, INV, true>(x, tw, hprefix, s_pass, sg0, q, qinv, every2);
        else
            fp_butterflies<R, INV, false>(x, tw, hprefix, s_pass, sg0, q, qinv, every2);
        if (io.gdst) {
#pragma unroll
            for (int m = 0; m < E; m++) {
                const double y = INV ? fmulmod(x[m], ninv_f, q, qinv) : x[m];
                io.gdst[base + ((u32)m << low_bits)] = to_canon(y, q, qinv);
            }
        } else {
#pragma unroll
            for (int m = 0; m < E; m++) lds[pad(base + ((u32)m << low_bits))] = fbal(x[m], q, qinv);
        }
    }
}

template <bool INV, int THREADS, bool R5>
__device__ __forceinline__ void run_round_fp(u32 r, double* lds, const double* tw, double q,
                                             double qinv, bool every2, u32 log_g, u32 log_c,
                                             u32 sg0, u32 s_pass, u32 g0, u32 lo_bits, RoundIO io,
                                             double ninv_f)
{
#define VR_FP_ROUND(RR)                                                                              \
    ntt_round_fp<RR, INV, THREADS>(lds, tw, q, qinv, every2, log_g, log_c, sg0, s_pass, g0, lo_bits, \
                                   io, ninv_f)
    switch (r) {
    case 5:
        if constexpr (R5) VR_FP_ROUND(5);
        break;
    case 4: VR_FP_ROUND(4); break;
    case 3: VR_FP_ROUND(3); break;
    case 2: VR_FP_ROUND(2); break;
    default: VR_FP_ROUND(1); break;
    }
#undef VR_FP_ROUND
}

template <bool INV, int THREADS, bool R5>
__device__ __forceinline__ void run_round(u32 r, u64* lds, const u64* tw, const ModQ& mq, u32 log_g,
                                          u32 log_c, u32 sg0, u32 s_pass, u32 g0, u32 lo_bits,
                                          RoundIO io)
{
    switch (r) {
    case 5:
        // the integer butterflies would spill with 32 words per thread: four
        // stages, then one (the block is uniformly on this path)
        if constexpr (R5) {
            RoundIO a = io, b = io;
            a.gdst = nullptr;
            b.gsrc = nullptr;
            if (!INV) {
                ntt_round<4, INV, THREADS>(lds, tw, mq, log_g, log_c, sg0, s_pass, g0, lo_bits, a);
                __syncthreads();
                ntt_round<1, INV, THREADS>(lds, tw, mq, log_g, log_c, sg0 + 4, s_pass, g0, lo_bits, b);
            } else {
                ntt_round<4, INV, THREADS>(lds, tw, mq, log_g, log_c, sg0 + 1, s_pass, g0, lo_bits, a);
                __syncthreads();
                ntt_round<1, INV, THREADS>(lds, tw, mq, log_g, log_c, sg0, s_pass, g0, lo_bits, b);
            }
        }
        break;
    case 4: ntt_round<4, INV, THREADS>(lds, tw, mq, log_g, log_c, sg0, s_pass, g0, lo_bits, io); break;
    case 3: ntt_round<3, INV, THREADS>(lds, tw, mq, log_g, log_c, sg0, s_pass, g0, lo_bits, io); break;
    case 2: ntt_round<2, INV, THREADS>(lds, tw, mq, log_g, log_c, sg0, s_pass, g0, lo_bits, io); break;
    default: ntt_round<1, INV, THREADS>(lds, tw, mq, log_g, log_c, sg0, s_pass, g0, lo_bits, io); break;
    }
}

template <int THREADS, bool INV, bool DIRECT, bool R5>
__global__ __launch_bounds__(THREADS) void k_ntt_pass(NttPass p)
{
    extern __shared__ u64 lds[];
    const u32 n = 1u << p.log_n;
    const u32 G = 1u << p.log_g;
    const u32 C = 1u << p.log_c;
    const u32 tile = G << p.log_c;
    const u32 lo_bits = p.log_n - p.s0 - p.log_g;
    const u32 blocks_per_limb = (n >> p.log_g) >> p.log_c;
    const u32 rl = blockIdx.x / blocks_per_limb;
    const u32 g0 = (blockIdx.x - rl * blocks_per_limb) << p.log_c;
    const u32 r = limb_order(p.ls, p.r0 + rl);

    const u64* src;
    u64* dst;
    u32 mod;
    limb_addr(p.ls, r, n, p.L, &src, &dst, &mod);
    if (!p.first) src = dst;
    const ModQ m = p.mq[mod];
    const u64 q = m.q, q2 = 2 * m.q;
    const bool fp = q < (1ull << 51);   // uniform over the workgroup (one limb)
    const double qd = (double)q, qinv = 1.0 / qd;
    // fused one-limb base conversion: this limb's source and its modulus
    u64 cq = 0;
    if (!INV && p.first && p.ls.cv_src) {
        const u32 poly = r / p.ls.per_poly;
        const u32 ct = poly / p.ls.cv_beta, d = poly - ct * p.ls.cv_beta;
        src = p.ls.cv_src + (size_t)ct * p.ls.cv_ct_stride + (size_t)d * n;
        cq = p.mq[p.ls.cv_mod0 + d].q;
    }

    // a pass over the whole limb reads and writes global memory in its first
    // and last round; other passes stage the tile through LDS with coalesced loads
    const bool direct = DIRECT;   // launched only for a single pass over the whole limb
    const bool strided = lo_bits > 0;
    // tile word e <-> (column c, row v) and its global index
    auto locate = [&](u32 e, u32* slot) -> size_t {
        u32 c, v;
        if (strided) { v = e >> p.log_c; c = e & (C - 1); }
        else { c = e >> p.log_g; v = e & (G - 1); }
        const u32 g = g0 + c;
        const u32 H = g >> lo_bits, Lo = g & ((1u << lo_bits) - 1);
        *slot = pad(c * G + v);
        return ((size_t)H << (p.log_n - p.s0)) + ((size_t)v << lo_bits) + Lo;
    };
    if (!direct) {
        // kBatch loads in flight per thread before the first one is consumed
        for (u32 e0 = threadIdx.x; e0 < tile; e0 += kBatch * THREADS) {
            u64 x[kBatch];
            u32 slot[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; j++) {
                const u32 e = e0 + j * THREADS;
                const size_t idx = locate(e < tile ? e : e0, &slot[j]);
                x[j] = e < tile ? src[idx] : 0;
            }
#pragma unroll
            for (int j = 0; j < kBatch; j++) {
                if (e0 + j * THREADS >= tile) break;
                u64 v = x[j];
                if (cq) v = conv_one(v, cq, q, m.one_s);
                // first pass of the FP64 path: canonical uint64 -> balanced double;
                // later passes read the balanced doubles the previous pass stored
                if (fp && p.first) v = __double_as_longlong(to_bal(v, q, qd));
                lds[slot[j]] = v;
            }
        }
        __syncthreads();
    }
    const double ninv_f = m.ninv > q / 2 ? -(double)(q - m.ninv) : (double)m.ninv;

    if (fp) {
        double* ldf = (double*)lds;
        const double* twf = p.twf + (size_t)mod * n;
        const bool every2 = q >= (1ull << 50);
        if (!INV) {
            for (u32 sg0 = 0; sg0 < p.log_g;) {
                u32 rr = p.log_g - sg0 < p.max_r ? p.log_g - sg0 : p.max_r;
                RoundIO io;
                if (direct && sg0 == 0) io.gsrc = src, io.cq = cq, io.t_one_s = m.one_s;
                if (direct && sg0 + rr == p.log_g) io.gdst = dst;
                run_round_fp<false, THREADS, R5>(rr, ldf, twf, qd, qinv, every2, p.log_g, p.log_c, sg0,
                                             p.s0, g0, lo_bits, io, ninv_f);
                sg0 += rr;
                __syncthreads();
            }
        } else {
            for (u32 top = p.log_g; top > 0;) {
                u32 rr = top < p.max_r ? top : p.max_r;
                RoundIO io;
                if (direct && top == p.log_g) io.gsrc = src;
                if (direct && top == rr) io.gdst = dst;
                run_round_fp<true, THREADS, R5>(rr, ldf, twf, qd, qinv, true, p.log_g, p.log_c, top - rr,
                                            p.s0, g0, lo_bits, io, ninv_f);
                top -= rr;
                __syncthreads();
            }
        }
    } else {
        const u64* tw = p.tw + (size_t)mod * n * 2;
        if (!INV) {
            for (u32 sg0 = 0; sg0 < p.log_g;) {
                u32 rr = p.log_g - sg0 < p.max_r ? p.log_g - sg0 : p.max_r;
                RoundIO io;
                if (direct && sg0 == 0) io.gsrc = src, io.cq = cq, io.t_one_s = m.one_s;
                if (direct && sg0 + rr == p.log_g) io.gdst = dst;
                run_round<false, THREADS, R5>(rr, lds, tw, m, p.log_g, p.log_c, sg0, p.s0, g0, lo_bits, io);
                sg0 += rr;
                __syncthreads();
            }
        } else {
            for (u32 top = p.log_g; top > 0;) {
                u32 rr = top < p.max_r ? top : p.max_r;
                RoundIO io;
                if (direct && top == p.log_g) io.gsrc = src;
                if (direct && top == rr) io.gdst = dst;
                run_round<true, THREADS, R5>(rr, lds, tw, m, p.log_g, p.log_c, top - rr, p.s0, g0, lo_bits,
                                         io);
                top -= rr;
                __syncthreads();
            }
        }
    }
    if (direct) return;

    for (u32 e0 = threadIdx.x; e0 < tile; e0 += kBatch * THREADS) {
        u64 xs[kBatch];
        size_t gi[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; j++) {
            const u32 e = e0 + j * THREADS;
            u32 slot;
            gi[j] = locate(e < tile ? e : e0, &slot);
            xs[j] = lds[slot];
        }
#pragma unroll
        for (int j = 0; j < kBatch; j++) {
            if (e0 + j * THREADS >= tile) break;
            const size_t idx = gi[j];
            u64 x = xs[j];
            if (fp) {
                if (p.last) {
                    double y = __longlong_as_double(x);
                    if (INV) y = fmulmod(y, ninv_f, qd, qinv);
                    x = to_canon(y, qd, qinv);
                }
            } else if (p.last) {
                if (!INV) {
                    x = x >= q2 ? x - q2 : x;
                    x = x >= q ? x - q : x;
                } else {
                    x = shoup(x, m.ninv, m.ninv_s, q);
                }
            }
            dst[idx] = x;
        }
    }
}

// ---------------------------------------------------------------------------
// Whole-limb transform with the round geometry fixed at compile time.
//
// One workgroup of 2^(LOGN - LOGE) threads transforms one limb of 2^LOGN
// words, each thread holding 2^LOGE words per round.  The rounds (LOGE stages
// each, the last one taking the remainder) are unrolled at compile time, so
// every shift, mask and offset is a constant: the words of a group differ
// only in index bits [lb, lb + R), which the group's base leaves clear, hence
// pad(base | m << lb) = pad(base) + pad(m << lb) and each word's LDS address
// is one per-group register plus an immediate.  The first round reads global
// memory and the last writes it, so LDS is only visited between rounds.
//
// FP64 limbs (q < 2^51) reduce no more often than their bounds require (the
// bounds are those of the general kernel above: a product is within about
// q + |e| of zero, e the exact low part, |e| < q / 16 in every case below):
//   forward  q < 2^44: never before the final store (16 stages from |x| <=
//            q/2 stay below 26 q < 2^49); q < 2^50: every 4 stages; else 2;
//   inverse  q < 2^46: every 4 stages (sums at most double per stage: below
//            8.8 q); else every 2.
// The inverse's N^-1 is folded into its last stage, whose single twiddle w1
// becomes the two constants N^-1 and w1 N^-1 (one product per output word
// instead of a product for the stage and one for the scaling).

constexpr u32 padc(u32 i) { return i + (i >> 4); }

template <int LOGN, int LOGE>
struct LimbShape {
    static constexpr int T_LOG = LOGN - LOGE;
    static constexpr u32 T = 1u << T_LOG;
    static constexpr int NR = (LOGN + LOGE - 1) / LOGE;
    // forward round i covers stages [i LOGE, i LOGE + R(i))
    static constexpr int R(int i) { return (i + 1) * LOGE <= LOGN ? LOGE : LOGN - i * LOGE; }
};

// Forward FP64 butterflies of one group: global stages SG0 .. SG0 + R - 1,
// reducing after each stage s with (s + 1) % RED == 0 (RED = 0: never).
template <int LOGN, int R, int SG0, int RED, bool UNI>
__device__ __forceinline__ void limb_fp_fwd(double (&x)[1 << R], const double* tw, u32 hi, double q,
                                            double qinv)
{
    constexpr int E = 1 << R;
    if (UNI) hi = __builtin_amdgcn_readfirstlane(hi);
#pragma unroll
    for (int k = 0; k < R; k++) {
        const int half = 1 << (R - 1 - k);
        const double* twk = tw + (1u << (SG0 + k)) + (hi << k);
#pragma unroll
        for (int j = 0; j < (1 << k); j++) {
            const double w = twk[j];
#pragma unroll
            for (int i = 0; i < half; i++) {
                const int m1 = (j << (R - k)) + i, m2 = m1 + half;
                const double X = x[m1];
                const double T = fmulmod(x[m2], w, q, qinv);
                x[m1] = X + T;
                x[m2] = X - T;
            }
        }
        const int s = SG0 + k;
        if (RED && (s + 1) % (RED ? RED : 1) == 0 && s != LOGN - 1) {
#pragma unroll
            for (int m = 0; m < E; m++) x[m] = fbal(x[m], q, qinv);
        }
    }
}

// Inverse FP64 butterflies: stages SG0 + R - 1 down to SG0; stage 0 takes
// the folded constants (n1 = N^-1, w1n = w1 N^-1).
template <int LOGN, int R, int SG0, int RED, bool UNI>
__device__ __forceinline__ void limb_fp_inv(double (&x)[1 << R], const double* tw, u32 hi, double q,
                                            double qinv, double n1, double w1n)
{
    constexpr int E = 1 << R;
    if (UNI) hi = __builtin_amdgcn_readfirstlane(hi);
#pragma unroll
    for (int k = R - 1; k >= 0; k--) {
        const int half = 1 << (R - 1 - k);
        const int s = SG0 + k;
        const double* twk = tw + (1u << s) + (hi << k);
#pragma unroll
        for (int j = 0; j < (1 << k); j++) {
#pragma unroll
            for (int i = 0; i < half; i++) {
                const int m1 = (j << (R - k)) + i, m2 = m1 + half;
                const double X = x[m1], Y = x[m2];
                if (s == 0) {
                    x[m1] = fmulmod(X + Y, n1, q, qinv);
                    x[m2] = fmulmod(X - Y, w1n, q, qinv);
                } else {
                    x[m1] = X + Y;
                    x[m2] = fmulmod(X - Y, twk[j], q, qinv);
                }
            }
        }
        if (RED && (LOGN - s) % (RED ? RED : 1) == 0 && s != 0) {
#pragma unroll
            for (int m = 0; m < E; m++) x[m] = fbal(x[m], q, qinv);
        }
    }
}

// Integer (Shoup, lazy) butterflies with the same compile-time geometry:
// forward values in [0, 4q), inverse in [0, 2q); stage 0 of the inverse
// takes the folded constants as (w, w') pairs.
template <int R, int SG0, bool INV, bool UNI>
__device__ __forceinline__ void limb_int(u64 (&x)[1 << R], const ulonglong2* tw, u32 hi, u64 q,
                                         ulonglong2 n1, ulonglong2 w1n)
{
    if (UNI) hi = __builtin_amdgcn_readfirstlane(hi);
    const u64 q2 = 2 * q;
    if (!INV) {
#pragma unroll
        for (int k = 0; k < R; k++) {
            const int half = 1 << (R - 1 - k);
            const ulonglong2* twk = tw + (1u << (SG0 + k)) + (hi << k);
#pragma unroll
            for (int j = 0; j < (1 << k); j++) {
                const ulonglong2 t = twk[j];
#pragma unroll
                for (int i = 0; i < half; i++) {
                    const int m1 = (j << (R - k)) + i, m2 = m1 + half;
                    u64 X = x[m1];
                    X = X >= q2 ? X - q2 : X;
                    const u64 T = shoup_lazy(x[m2], t.x, t.y, q);
                    x[m1] = X + T;
                    x[m2] = X + q2 - T;
                }
            }
        }
    } else {
#pragma unroll
        for (int k = R - 1; k >= 0; k--) {
            const int half = 1 << (R - 1 - k);
            const int s = SG0 + k;
            const ulonglong2* twk = tw + (1u << s) + (hi << k);
#pragma unroll
            for (int j = 0; j < (1 << k); j++) {
#pragma unroll
                for (int i = 0; i < half; i++) {
                    const int m1 = (j << (R - k)) + i, m2 = m1 + half;
                    const u64 X = x[m1], Y = x[m2];
                    if (s == 0) {
                        x[m1] = shoup_lazy(X + Y, n1.x, n1.y, q);
                        x[m2] = shoup_lazy(X + q2 - Y, w1n.x, w1n.y, q);
                    } else {
                        const ulonglong2 t = twk[j];
                        const u64 S = X + Y;
                        x[m1] = S >= q2 ? S - q2 : S;
                        x[m2] = shoup_lazy(X + q2 - Y, t.x, t.y, q);
                    }
                }
            }
        }
    }
}

// Per-limb constants of the whole-limb kernel.
struct LimbK {
    u32 tid;    // threadIdx.x
    const u64* src;
    u64* dst;
    const u64* tw64;
    const double* twf;
    u64 q, cq, one_s;
    double qd, qinv, n1f, w1nf;
    ulonglong2 n1, w1n;
    // forward epilogue (ea != null): this limb's rows of A, of the output and
    // of B (eb_g: Galois element B is read through), and its scaling
    const u64* ea;
    u64* eo;
    const u64* eb;
    u32 eb_g;
    ulonglong2 ec;
    double ecf;
    bool ebm;          // B is scaled by ebc before it is added
    ulonglong2 ebc;
    double ebcf;
};

// Where limb r's input comes from: the limb itself, or (forward, fused
// conversion) the one-limb source it is converted from, modulo *cq.
template <int LOGN, bool INV>
__device__ __forceinline__ const u64* limb_src(const NttPass& p, u32 r, u64** dst, u32* mod, u64* cq)
{
    constexpr u32 n = 1u << LOGN;
    const u64* src;
    limb_addr(p.ls, r, n, p.L, &src, dst, mod);
    *cq = 0;
    if (!INV && p.ls.cv_src) {
        const u32 poly = r / p.ls.per_poly;
        const u32 ct = poly / p.ls.cv_beta, d = poly - ct * p.ls.cv_beta;
        src = p.ls.cv_src + (size_t)ct * p.ls.cv_ct_stride + (size_t)d * n;
        *cq = p.mq[p.ls.cv_mod0 + d].q;
    }
    return src;
}

template <int LOGN, bool INV>
__device__ __forceinline__ LimbK limb_consts(const NttPass& p, u32 r)
{
    constexpr u32 n = 1u << LOGN;
    LimbK c;
    u32 mod;
    c.src = limb_src<LOGN, INV>(p, r, &c.dst, &mod, &c.cq);
    const ModQ& mq = p.mq[mod];
    c.q = mq.q;
    c.one_s = mq.one_s;
    c.tw64 = p.tw + (size_t)mod * n * 2;
    c.twf = p.twf + (size_t)mod * n;
    c.n1 = make_ulonglong2(mq.ninv, mq.ninv_s);
    c.w1n = make_ulonglong2(mq.inw1, mq.inw1_s);
    c.qd = (double)c.q;
    c.qinv = 1.0 / c.qd;
    c.n1f = to_bal(mq.ninv, c.q, c.qd);
    c.w1nf = to_bal(mq.inw1, c.q, c.qd);
    c.ea = nullptr;
    if (!INV && p.ls.epi.a) {
        const NttEpilogue& ep = p.ls.epi;
        const u32 poly = r / p.ls.per_poly, i = r - poly * p.ls.per_poly;
        const u32 k = poly >> 1, j = poly & 1;
        c.ea = ep.a + k * ep.a_ct + j * ep.a_comp + (size_t)i * n;
        c.eo = (j ? ep.out1 : ep.out0) + k * ep.out_ct + (size_t)i * n;
        const u64* add = j ? ep.add1 : ep.add0;
        c.eb = add ? add + k * ep.add_ct + (size_t)i * n : nullptr;
        c.eb_g = j ? 1 : ep.add0_g;
        c.ec = ep.cmul[mod];
        c.ecf = to_bal(c.ec.x, c.q, c.qd);
        c.ebm = ep.bmul != nullptr;
        if (c.ebm) {
            c.ebc = ep.bmul[mod];
            c.ebcf = to_bal(c.ebc.x, c.q, c.qd);
        }
    }
    return c;
}

// LDS words written by lanes of this wave are visible to its other lanes
// (LDS executes one wave's instructions in order; the fences keep the
// compiler from moving the accesses across).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The finish of a forward transform on one word: (A - y) c (+ B, or + B c_b)
// with B read through the Galois map, FP64 path (|A - y| < 27 q, the product
// within 1.5 q, 3 q when q >= 2^50, reduced before B is added) or integer path
// (y lazy in [0, 4q)).
__device__ __forceinline__ u64 finish_fp(const LimbK& c, u64 a, u64 b, double y)
{
    double v = fbal(fmulmod(to_bal(a, c.q, c.qd) - y, c.ecf, c.qd, c.qinv), c.qd, c.qinv);
    if (c.eb) {
        double bb = to_bal(b, c.q, c.qd);
        if (c.ebm) bb = fbal(fmulmod(bb, c.ebcf, c.qd, c.qinv), c.qd, c.qinv);
        v += bb;
    }
    return to_canon(v, c.qd, c.qinv);
}

__device__ __forceinline__ u64 finish_int(const LimbK& c, u64 a, u64 b, u64 y)
{
    const u64 q = c.q, q2 = 2 * q;
    y = y >= q2 ? y - q2 : y;
    y = y >= q ? y - q : y;
    u64 v = shoup(a + q - y, c.ec.x, c.ec.y, q);
    if (c.eb) v = add_mod(v, c.ebm ? shoup(b, c.ebc.x, c.ebc.y, q) : b, q);
    return v;
}

// Round i's geometry: R stages from global stage SG0, groups of 2^R words at
// index stride 2^LB, GPT groups per thread.
template <int LOGN, int LOGE, int I>
struct RoundShape {
    using S = LimbShape<LOGN, LOGE>;
    static constexpr int R = S::R(I);
    static constexpr int SG0 = I * LOGE;
    static constexpr int E = 1 << R;
    static constexpr int LB = LOGN - SG0 - R;
    static constexpr int GPT = 1 << (LOGE - R);
};

// Forward round I (or inverse round I, walking the forward rounds from the
// last) over the thread's groups.  FP = the limb is on the FP64 path.
template <int LOGN, int LOGE, int I, bool INV, bool FP, int RED>
__device__ __forceinline__ void limb_round(u64* lds, const LimbK& c)
{
    using S = LimbShape<LOGN, LOGE>;
    using G = RoundShape<LOGN, LOGE, I>;
    constexpr int R = G::R, SG0 = G::SG0, E = G::E, LB = G::LB, GPT = G::GPT;
    constexpr bool UNI = LB >= 6;
    // the forward transform's first round and the inverse's last face the
    // limb's coefficients in global memory; so do the forward's last and the
    // inverse's first
    constexpr bool FROM_G = INV ? (I == S::NR - 1) : (I == 0);
    constexpr bool TO_G = INV ? (I == 0) : (I == S::NR - 1);
    // groups of consecutive words (the forward's last round, the inverse's
    // first): global memory is accessed across lanes instead, each wave
    // staging its own 64 groups through their LDS words
    constexpr bool XPOSE = LB == 0;
    const u32 lane = c.tid & 63;
    double* ldf = (double*)lds;
#pragma unroll
    for (int g = 0; g < GPT; g++) {
        const u32 gid = c.tid + (u32)g * S::T;
        const u32 hi = gid >> LB, lo = gid & ((1u << LB) - 1);
        const u32 base = (hi << (LB + R)) | lo;
        const u32 pb = pad(base);
        const u32 rb = (gid - lane) * E;   // this wave's words when XPOSE
        // limb word of the m-th global access
        auto gword = [&](int m) -> u32 { return XPOSE ? rb + (u32)m * 64 + lane : base + ((u32)m << LB); };
        if constexpr (FP) {
            double x[E];
            if (FROM_G) {
                u64 v[E];
#pragma unroll
                for (int m = 0; m < E; m++) v[m] = c.src[gword(m)];
#pragma unroll
                for (int m = 0; m < E; m++) {
                    u64 t = v[m];
                    if (!INV && c.cq) t = conv_one(t, c.cq, c.q, c.one_s);
                    x[m] = to_bal(t, c.q, c.qd);
                }
                if constexpr (XPOSE) {
#pragma unroll
                    for (int m = 0; m < E; m++) ldf[pad(gword(m))] = x[m];
                    wave_lds_sync();
#pragma unroll
                    for (int m = 0; m < E; m++) x[m] = ldf[pb + m];
                }
            } else {
#pragma unroll
                for (int m = 0; m < E; m++) x[m] = ldf[pb + padc((u32)m << LB)];
            }
            if constexpr (INV)
                limb_fp_inv<LOGN, R, SG0, RED, UNI>(x, c.twf, hi, c.qd, c.qinv, c.n1f, c.w1nf);
            else
                limb_fp_fwd<LOGN, R, SG0, RED, UNI>(x, c.twf, hi, c.qd, c.qinv);
            if constexpr (TO_G) {
                if constexpr (XPOSE) {
#pragma unroll
                    for (int m = 0; m < E; m++) ldf[pb + m] = x[m];
                    wave_lds_sync();
#pragma unroll
                    for (int m = 0; m < E; m++) x[m] = ldf[pad(gword(m))];
                }
                if (!INV && c.ea) {
                    u64 av[E], bv[E];
#pragma unroll
                    for (int m = 0; m < E; m++) {
                        const u32 idx = gword(m);
                        av[m] = c.ea[idx];
                        if (c.eb) bv[m] = c.eb[c.eb_g != 1 ? galois_src(idx, c.eb_g, LOGN) : idx];
                    }
#pragma unroll
                    for (int m = 0; m < E; m++) c.eo[gword(m)] = finish_fp(c, av[m], bv[m], x[m]);
                } else {
#pragma unroll
                    for (int m = 0; m < E; m++) c.dst[gword(m)] = to_canon(x[m], c.qd, c.qinv);
                }
            } else {
#pragma unroll
                for (int m = 0; m < E; m++) ldf[pb + padc((u32)m << LB)] = x[m];
            }
        } else {
            const u64 q = c.q, q2 = 2 * q;
            u64 x[E];
            if (FROM_G) {
#pragma unroll
                for (int m = 0; m < E; m++) x[m] = c.src[gword(m)];
                if (!INV && c.cq) {
#pragma unroll
                    for (int m = 0; m < E; m++) x[m] = conv_one(x[m], c.cq, q, c.one_s);
                }
                if constexpr (XPOSE) {
#pragma unroll
                    for (int m = 0; m < E; m++) lds[pad(gword(m))] = x[m];
                    wave_lds_sync();
#pragma unroll
                    for (int m = 0; m < E; m++) x[m] = lds[pb + m];
                }
            } else {
#pragma unroll
                for (int m = 0; m < E; m++) x[m] = lds[pb + padc((u32)m << LB)];
            }
            limb_int<R, SG0, INV, UNI>(x, (const ulonglong2*)c.tw64, hi, q, c.n1, c.w1n);
            if constexpr (TO_G) {
                if constexpr (XPOSE) {
#pragma unroll
                    for (int m = 0; m < E; m++) lds[pb + m] = x[m];
                    wave_lds_sync();
#pragma unroll
                    for (int m = 0; m < E; m++) x[m] = lds[pad(gword(m))];
                }
                if (!INV && c.ea) {
                    u64 av[E], bv[E];
#pragma unroll
                    for (int m = 0; m < E; m++) {
                        const u32 idx = gword(m);
                        av[m] = c.ea[idx];
                        if (c.eb) bv[m] = c.eb[c.eb_g != 1 ? galois_src(idx, c.eb_g, LOGN) : idx];
                    }
#pragma unroll
                    for (int m = 0; m < E; m++) c.eo[gword(m)] = finish_int(c, av[m], bv[m], x[m]);
                } else {
#pragma unroll
                    for (int m = 0; m < E; m++) {
                        u64 y = x[m];
                        if (!INV) y = y >= q2 ? y - q2 : y;
                        c.dst[gword(m)] = y >= q ? y - q : y;
                    }
                }
            } else {
#pragma unroll
                for (int m = 0; m < E; m++) lds[pb + padc((u32)m << LB)] = x[m];
            }
        }
    }
}

// One word of each 128-byte line of a limb row per thread (2^LOGN / 16 lines).
template <int LOGN, int LOGE>
struct LinePrefetch {
    static constexpr u32 LINES = (1u << LOGN) / 16;
    static constexpr u32 PER = LINES > LimbShape<LOGN, LOGE>::T ? LINES / LimbShape<LOGN, LOGE>::T : 1;
    u64 a[PER], b[PER];
};

// Rounds I, I+1, ... (inverse: I, I-1, ...) with a barrier between rounds.
// A fused finish reads its operands in the last round; after the first
// round every thread loads one word of each of their 128-byte lines, so
// that the operands are in cache by then (the words are consumed at the
// kernel's end).
template <int LOGN, int LOGE, bool INV, bool FP, int RED, int I>
__device__ __forceinline__ void limb_rounds(u64* lds, const LimbK& c, LinePrefetch<LOGN, LOGE>& pf)
{
    using S = LimbShape<LOGN, LOGE>;
    using PF = LinePrefetch<LOGN, LOGE>;
    static_assert(S::NR >= 2, "whole-limb kernel needs two rounds or more");
    if constexpr (I >= 0 && I < S::NR) {
        if constexpr (!INV && I == 1) {
            if (c.ea) {
#pragma unroll
                for (u32 k = 0; k < PF::PER; k++) {
                    const u32 line = c.tid + k * S::T;
                    if (line < PF::LINES) {
                        pf.a[k] = c.ea[line * 16];
                        if (c.eb) pf.b[k] = c.eb[line * 16];
                    }
                }
            }
        }
        limb_round<LOGN, LOGE, I, INV, FP, RED>(lds, c);
        constexpr int NEXT = INV ? I - 1 : I + 1;
        if constexpr (NEXT >= 0 && NEXT < S::NR) {
            __syncthreads();
            limb_rounds<LOGN, LOGE, INV, FP, RED, NEXT>(lds, c, pf);
        }
    }
}

template <int LOGN, int LOGE, bool INV>
__device__ __forceinline__ void limb_transform(u64* lds, const LimbK& c, LinePrefetch<LOGN, LOGE>& pf)
{
    constexpr int I0 = INV ? LimbShape<LOGN, LOGE>::NR - 1 : 0;
    if (c.q < (1ull << 51)) {
        if (!INV) {
            if (c.q < (1ull << 44))
                limb_rounds<LOGN, LOGE, INV, true, 0, I0>(lds, c, pf);
            else if (c.q < (1ull << 50))
                limb_rounds<LOGN, LOGE, INV, true, 4, I0>(lds, c, pf);
            else
                limb_rounds<LOGN, LOGE, INV, true, 2, I0>(lds, c, pf);
        } else {
            if (c.q < (1ull << 46))
                limb_rounds<LOGN, LOGE, INV, true, 4, I0>(lds, c, pf);
            else
                limb_rounds<LOGN, LOGE, INV, true, 2, I0>(lds, c, pf);
        }
    } else {
        limb_rounds<LOGN, LOGE, INV, false, 4, I0>(lds, c, pf);
    }
}

// One workgroup per limb.  (A persistent variant, one workgroup per CU
// walking the limbs and pulling the next one into cache during the last
// round, measured slower: the hardware already starts the next workgroup as
// soon as the previous one frees the CU's LDS.)
template <int LOGN, int LOGE, bool INV>
__global__ __launch_bounds__(1u << (LOGN - LOGE)) void k_ntt_limb(NttPass p)
{
    extern __shared__ u64 lds[];
    LimbK c = limb_consts<LOGN, INV>(p, limb_order(p.ls, p.r0 + blockIdx.x));
    c.tid = threadIdx.x;
    LinePrefetch<LOGN, LOGE> pf;
    limb_transform<LOGN, LOGE, INV>(lds, c, pf);
    if (!INV && c.ea) {
#pragma unroll
        for (u32 k = 0; k < LinePrefetch<LOGN, LOGE>::PER; k++) {
            if (c.tid + k * LimbShape<LOGN, LOGE>::T < LinePrefetch<LOGN, LOGE>::LINES) {
                asm volatile("" ::"v"(pf.a[k]));
                if (c.eb) asm volatile("" ::"v"(pf.b[k]));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Two-pass transform with the round geometry fixed at compile time, for rings
// whose limb does not fit in one CU's LDS (N = 2^15, 2^16).
//
// Pass 0 runs global stages [0, A) on tiles of 2^LC consecutive columns: tile
// word e = v 2^LC + c is coefficient v 2^(LOGN - A) + col0 + c (v < 2^A), so
// each of a thread's loads and stores covers 2^LC consecutive words across
// neighbouring lanes.  Pass 1 runs stages [A, LOGN) on 2^LC consecutive
// blocks of 2^(LOGN - A) words: tile word e is coefficient tile0 + e.  Inside
// a pass the rounds are those of the whole-limb kernel (16 words per thread,
// four stages per round, the last taking the remainder): the first round
// reads global memory, the last writes it, and LDS is visited only between
// rounds.  A tile is 2^(P + LC) words (P = the pass's stages), small enough
// for several workgroups per CU, so that one workgroup's global loads and
// stores overlap the butterflies of another.
//
// Twiddle prefixes: at global stage s a butterfly's twiddle is indexed by its
// coefficient index >> (LOGN - s).  In pass 0 that is v >> (A - s), which is
// the group's hi below; in pass 1 it is (tile0 + e) >> (LOGN - s), i.e. hi
// plus tile0 >> (LOGN - s).  Between the passes the FP64 path stores its
// balanced doubles (exact integers, bounded as in a single pass since the
// reduction schedule follows the global stage), the integer path its lazy
// residues; only the transform's own input and output are canonical.
template <int LOGN, int A, int LC, int PASS>
struct SplitShape {
    static constexpr int P = PASS == 0 ? A : LOGN - A;   // stages in the pass
    static constexpr int LOGT = P + LC;                  // tile words (log)
    static constexpr u32 T = 1u << (LOGT - 4);           // 16 words per thread
    static constexpr int TOP = PASS == 0 ? LOGT : P;     // the pass pairs tile bits below TOP
    static constexpr int S0 = PASS == 0 ? 0 : A;         // global stage of the pass's first
    static constexpr int NR = (P + 3) / 4;
    static constexpr int R(int i) { return (i + 1) * 4 <= P ? 4 : P - i * 4; }
    static constexpr int WG_LOG = LOGN - LOGT;           // workgroups per limb (log)
};

// coefficient index of tile word e in tile wg
template <int LOGN, int A, int LC, int PASS>
__device__ __forceinline__ u32 split_addr(u32 e, u32 wg)
{
    if constexpr (PASS == 0)
        return ((e >> LC) << (LOGN - A)) + (wg << LC) + (e & ((1u << LC) - 1));
    else
        return (wg << (LOGN - A + LC)) + e;
}

// words whose finish operands a thread loads together in the last round
constexpr int kFinBatch = 4;

template <int LOGN, int A, int LC, int PASS, int I, bool INV, bool FP, int RED>
__device__ __forceinline__ void split_round(u64* lds, const LimbK& c, u32 wg)
{
    using S = SplitShape<LOGN, A, LC, PASS>;
    constexpr int R = S::R(I), SGL = 4 * I, SG0 = S::S0 + SGL, E = 1 << R;
    constexpr int LB = S::TOP - SGL - R, GPT = 1 << (4 - R);
    constexpr bool UNI = LB >= 6;
    constexpr bool FROM_G = INV ? (I == S::NR - 1) : (I == 0);
    constexpr bool TO_G = INV ? (I == 0) : (I == S::NR - 1);
    // the pass launched first reads the canonical input, the second writes
    // the canonical output; in between the intermediate form
    constexpr bool FIRST = INV ? PASS == 1 : PASS == 0;
    // groups of consecutive words (pass 1's last forward round, first
    // inverse one): global memory is accessed across lanes instead, each
    // wave staging its own 64 groups through their LDS words
    constexpr bool XPOSE = LB == 0;
    const u32 hoff = PASS == 1 ? wg << (LC + SGL) : 0u;
    constexpr int FB = E < kFinBatch ? E : kFinBatch;
    const u32 lane = c.tid & 63;
    double* ldf = (double*)lds;
#pragma unroll
    for (int g = 0; g < GPT; g++) {
        const u32 gid = c.tid + (u32)g * S::T;
        const u32 hi = gid >> LB, lo = gid & ((1u << LB) - 1);
        const u32 base = (hi << (LB + R)) | lo;
        const u32 pb = pad(base);
        const u32 rb = (gid - lane) * E;   // this wave's words when XPOSE
        // tile word of the m-th global access
        auto gword = [&](int m) -> u32 { return XPOSE ? rb + (u32)m * 64 + lane : base + ((u32)m << LB); };
        if constexpr (FP) {
            double x[E];
            if constexpr (FROM_G) {
                u64 v[E];
#pragma unroll
                for (int m = 0; m < E; m++) v[m] = c.src[split_addr<LOGN, A, LC, PASS>(gword(m), wg)];
#pragma unroll
                for (int m = 0; m < E; m++) {
                    if constexpr (FIRST) {
                        u64 t = v[m];
                        if (!INV && c.cq) t = conv_one(t, c.cq, c.q, c.one_s);
                        x[m] = to_bal(t, c.q, c.qd);
                    } else {
                        x[m] = __longlong_as_double(v[m]);
                    }
                }
                if constexpr (XPOSE) {
#pragma unroll
                    for (int m = 0; m < E; m++) ldf[pad(gword(m))] = x[m];
                    wave_lds_sync();
#pragma unroll
                    for (int m = 0; m < E; m++) x[m] = ldf[pb + m];
                }
            } else {
#pragma unroll
                for (int m = 0; m < E; m++) x[m] = ldf[pb + padc((u32)m << LB)];
            }
            if constexpr (INV)
                limb_fp_inv<LOGN, R, SG0, RED, UNI>(x, c.twf, hi + hoff, c.qd, c.qinv, c.n1f, c.w1nf);
            else
                limb_fp_fwd<LOGN, R, SG0, RED, UNI>(x, c.twf, hi + hoff, c.qd, c.qinv);
            if constexpr (TO_G) {
                if constexpr (XPOSE) {
#pragma unroll
                    for (int m = 0; m < E; m++) ldf[pb + m] = x[m];
                    wave_lds_sync();
#pragma unroll
                    for (int m = 0; m < E; m++) x[m] = ldf[pad(gword(m))];
                }
                if constexpr (FIRST) {
#pragma unroll
                    for (int m = 0; m < E; m++)
                        c.dst[split_addr<LOGN, A, LC, PASS>(gword(m), wg)] = __double_as_longlong(x[m]);
                } else if (!INV && c.ea) {
                    // the finish's operands in batches of kFinBatch words,
                    // so the pass keeps 4 waves per SIMD
#pragma unroll
                    for (int m0 = 0; m0 < E; m0 += FB) {
                        u64 av[FB], bv[FB];
#pragma unroll
                        for (int m = 0; m < FB; m++) {
                            const u32 idx = split_addr<LOGN, A, LC, PASS>(gword(m0 + m), wg);
                            av[m] = c.ea[idx];
                            if (c.eb) bv[m] = c.eb[c.eb_g != 1 ? galois_src(idx, c.eb_g, LOGN) : idx];
                        }
#pragma unroll
                        for (int m = 0; m < FB; m++) {
                            const u32 idx = split_addr<LOGN, A, LC, PASS>(gword(m0 + m), wg);
                            c.eo[idx] = finish_fp(c, av[m], bv[m], x[m0 + m]);
                        }
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < E; m++)
                        c.dst[split_addr<LOGN, A, LC, PASS>(gword(m), wg)] = to_canon(x[m], c.qd, c.qinv);
                }
            } else {
#pragma unroll
                for (int m = 0; m < E; m++) ldf[pb + padc((u32)m << LB)] = x[m];
            }
        } else {
            const u64 q = c.q, q2 = 2 * q;
            u64 x[E];
            if constexpr (FROM_G) {
#pragma unroll
                for (int m = 0; m < E; m++) x[m] = c.src[split_addr<LOGN, A, LC, PASS>(gword(m), wg)];
                if (FIRST && !INV && c.cq) {
#pragma unroll
                    for (int m = 0; m < E; m++) x[m] = conv_one(x[m], c.cq, q, c.one_s);
                }
                if constexpr (XPOSE) {
#pragma unroll
                    for (int m = 0; m < E; m++) lds[pad(gword(m))] = x[m];
                    wave_lds_sync();
#pragma unroll
                    for (int m = 0; m < E; m++) x[m] = lds[pb + m];
                }
            } else {
#pragma unroll
                for (int m = 0; m < E; m++) x[m] = lds[pb + padc((u32)m << LB)];
            }
            limb_int<R, SG0, INV, UNI>(x, (const ulonglong2*)c.tw64, hi + hoff, q, c.n1, c.w1n);
            if constexpr (TO_G) {
                if constexpr (XPOSE) {
#pragma unroll
                    for (int m = 0; m < E; m++) lds[pb + m] = x[m];
                    wave_lds_sync();
#pragma unroll
                    for (int m = 0; m < E; m++) x[m] = lds[pad(gword(m))];
                }
                if constexpr (FIRST) {
#pragma unroll
                    for (int m = 0; m < E; m++) c.dst[split_addr<LOGN, A, LC, PASS>(gword(m), wg)] = x[m];
                } else if (!INV && c.ea) {
#pragma unroll
                    for (int m0 = 0; m0 < E; m0 += FB) {
                        u64 av[FB], bv[FB];
#pragma unroll
                        for (int m = 0; m < FB; m++) {
                            const u32 idx = split_addr<LOGN, A, LC, PASS>(gword(m0 + m), wg);
                            av[m] = c.ea[idx];
                            if (c.eb) bv[m] = c.eb[c.eb_g != 1 ? galois_src(idx, c.eb_g, LOGN) : idx];
                        }
#pragma unroll
                        for (int m = 0; m < FB; m++)
                            c.eo[split_addr<LOGN, A, LC, PASS>(gword(m0 + m), wg)] =
                                finish_int(c, av[m], bv[m], x[m0 + m]);
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < E; m++) {
                        u64 y = x[m];
                        if (!INV) y = y >= q2 ? y - q2 : y;
                        c.dst[split_addr<LOGN, A, LC, PASS>(gword(m), wg)] = y >= q ? y - q : y;
                    }
                }
            } else {
#pragma unroll
                for (int m = 0; m < E; m++) lds[pb + padc((u32)m << LB)] = x[m];
            }
        }
    }
}

template <int LOGN, int A, int LC, int PASS, bool INV, bool FP, int RED, int I>
__device__ __forceinline__ void split_rounds(u64* lds, const LimbK& c, u32 wg)
{
    using S = SplitShape<LOGN, A, LC, PASS>;
    if constexpr (I >= 0 && I < S::NR) {
        split_round<LOGN, A, LC, PASS, I, INV, FP, RED>(lds, c, wg);
        constexpr int NEXT = INV ? I - 1 : I + 1;
        if constexpr (NEXT >= 0 && NEXT < S::NR) {
            __syncthreads();
            split_rounds<LOGN, A, LC, PASS, INV, FP, RED, NEXT>(lds, c, wg);
        }
    }
}

// One workgroup per tile; the reduction schedule of the whole-limb kernel
// (its bounds cover 16 stages).
template <int LOGN, int A, int LC, int PASS, bool INV>
__global__ __launch_bounds__((SplitShape<LOGN, A, LC, PASS>::T)) void k_ntt_split(NttPass p)
{
    using S = SplitShape<LOGN, A, LC, PASS>;
    extern __shared__ u64 lds[];
    const u32 r = limb_order(p.ls, p.r0 + (blockIdx.x >> S::WG_LOG)), wg = blockIdx.x & ((1u << S::WG_LOG) - 1);
    LimbK c = limb_consts<LOGN, INV>(p, r);
    c.tid = threadIdx.x;
    constexpr bool FIRST = INV ? PASS == 1 : PASS == 0;
    if (!FIRST) {
        c.src = c.dst;
        c.cq = 0;
    }
    if (INV || PASS == 0) c.ea = nullptr;
    constexpr int I0 = INV ? S::NR - 1 : 0;
    if (c.q < (1ull << 51)) {
        if (!INV) {
            if (c.q < (1ull << 44))
                split_rounds<LOGN, A, LC, PASS, INV, true, 0, I0>(lds, c, wg);
            else if (c.q < (1ull << 50))
                split_rounds<LOGN, A, LC, PASS, INV, true, 4, I0>(lds, c, wg);
            else
                split_rounds<LOGN, A, LC, PASS, INV, true, 2, I0>(lds, c, wg);
        } else {
            if (c.q < (1ull << 46))
                split_rounds<LOGN, A, LC, PASS, INV, true, 4, I0>(lds, c, wg);
            else
                split_rounds<LOGN, A, LC, PASS, INV, true, 2, I0>(lds, c, wg);
        }
    } else {
        split_rounds<LOGN, A, LC, PASS, INV, false, 4, I0>(lds, c, wg);
    }
}

namespace {

constexpr u32 kSplitChunkDefault = 0;

struct PassCfg {
    u32 s0, log_g, log_c;
    u32 direct = 0;    // 1: whole-limb pass with global first/last rounds; 2: the same
                       // with the round geometry fixed at compile time; 3: a pass of
                       // the compile-time two-pass kernels
    u32 div = 16;      // tile words per thread
    u32 max_r = 4;     // stages per round
};

std::vector<PassCfg> default_plan(u32 log_n)
{
    if (log_n <= 14) return {{0, log_n, 0}};
    if (log_n == 15) return {{0, 7, 5}, {7, 8, 4}};
    return {{0, 8, 4}, {8, 8, 4}};   // 2^16
}

// Plans the autotuner times: the single LDS-resident pass where the limb
// fits, two-pass splits a + b = log N with 2^(3..7) groups per workgroup
// (tiles of 2^10 .. 2^14 words), and at 2^15 and 2^16 the compile-time
// two-pass kernels (listed last, so they are kept only when clearly faster).
std::vector<std::vector<PassCfg>> candidates(u32 log_n)
{
    std::vector<std::vector<PassCfg>> out;
    if (log_n <= 14) {
        out.push_back({{0, log_n, 0}});
        if (log_n >= 10) {
            if (log_n <= 13) out.push_back({{0, log_n, 0, 1, 16}});
            out.push_back({{0, log_n, 0, 1, 32}});
            if (log_n >= 13) out.push_back({{0, log_n, 0, 1, 32, 5}});   // rounds of five stages
            if (log_n >= 13) {
                // compile-time whole-limb kernels, 16 or 32 words per thread
                out.push_back({{0, log_n, 0, 2, 16}});
                out.push_back({{0, log_n, 0, 2, 32}});
            }
        }
    }
    if (log_n < 10) return out;
    for (u32 a = log_n / 2 - 1; a <= (log_n + 1) / 2 + 1; a++) {
        const u32 b = log_n - a;
        for (u32 c = 3; c <= 7; c++) {
            const u32 c1 = c, c2 = c;
            if (a + c1 < 10 || a + c1 > 14 || b + c2 < 10 || b + c2 > 14) continue;
            if (c1 > log_n - a || c2 > log_n - b) continue;
            out.push_back({{0, a, c1}, {a, b, c2}});
        }
    }
    if (log_n == 15 || log_n == 16) {
        // compile-time two-pass kernels: stages split a + b, 2^lc columns
        // (pass 0) or blocks (pass 1) per workgroup
        for (u32 a = log_n / 2; a <= (log_n + 1) / 2; a++)
            for (u32 lc = (log_n == 16 ? 3 : 4); lc <= 5; lc++)
                out.push_back({{0, a, lc, 3, 16}, {a, log_n - a, lc, 3, 16}});
    }
    return out;
}

template <int T, bool INV, bool DIRECT, bool R5 = false>
void launch_kernel(const NttPass& p, u32 blocks, size_t shmem, hipStream_t s)
{
    static std::once_flag attr;
    std::call_once(attr, [] {
        (void)hipFuncSetAttribute((const void*)k_ntt_pass<T, INV, DIRECT, R5>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    });
    hipLaunchKernelGGL((k_ntt_pass<T, INV, DIRECT, R5>), dim3(blocks), dim3(T), shmem, s, p);
}

template <int LOGN, int LOGE, bool INV>
void launch_limb(const NttPass& p, u32 n_limbs, hipStream_t s)
{
    static std::once_flag attr;
    const size_t shmem = (size_t)padc(1u << LOGN) * sizeof(u64);
    std::call_once(attr, [&] {
        (void)hipFuncSetAttribute((const void*)k_ntt_limb<LOGN, LOGE, INV>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    });
    hipLaunchKernelGGL((k_ntt_limb<LOGN, LOGE, INV>), dim3(n_limbs), dim3(1u << (LOGN - LOGE)), shmem, s, p);
}

template <int LOGN, int A, int LC, int PASS, bool INV>
void launch_split(const NttPass& p, u32 n_limbs, hipStream_t s)
{
    using S = SplitShape<LOGN, A, LC, PASS>;
    static std::once_flag attr;
    const size_t shmem = (size_t)padc(1u << S::LOGT) * sizeof(u64);
    std::call_once(attr, [&] {
        (void)hipFuncSetAttribute((const void*)k_ntt_split<LOGN, A, LC, PASS, INV>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    });
    hipLaunchKernelGGL((k_ntt_split<LOGN, A, LC, PASS, INV>), dim3(n_limbs << S::WG_LOG), dim3(S::T), shmem,
                       s, p);
}

template <bool INV>
void launch_pass(const NttPass& p, const PassCfg& c, u32 n_limbs, hipStream_t s)
{
    if (c.direct == 3) {
        // pass 0 starts at stage 0 and runs a = log_g stages; pass 1 starts at a
        const u32 pass = c.s0 == 0 ? 0 : 1;
        const u32 a = pass == 0 ? c.log_g : c.s0;
        if (c.div != 16 || (pass == 1 && a + c.log_g != p.log_n))
            throw Error(VR_EINVAL, "ntt: malformed two-pass plan");
        switch (p.log_n * 1000 + a * 100 + c.log_c * 10 + pass) {
        case 16830: launch_split<16, 8, 3, 0, INV>(p, n_limbs, s); break;
        case 16831: launch_split<16, 8, 3, 1, INV>(p, n_limbs, s); break;
        case 16840: launch_split<16, 8, 4, 0, INV>(p, n_limbs, s); break;
        case 16841: launch_split<16, 8, 4, 1, INV>(p, n_limbs, s); break;
        case 16850: launch_split<16, 8, 5, 0, INV>(p, n_limbs, s); break;
        case 16851: launch_split<16, 8, 5, 1, INV>(p, n_limbs, s); break;
        case 15740: launch_split<15, 7, 4, 0, INV>(p, n_limbs, s); break;
        case 15741: launch_split<15, 7, 4, 1, INV>(p, n_limbs, s); break;
        case 15750: launch_split<15, 7, 5, 0, INV>(p, n_limbs, s); break;
        case 15751: launch_split<15, 7, 5, 1, INV>(p, n_limbs, s); break;
        case 15840: launch_split<15, 8, 4, 0, INV>(p, n_limbs, s); break;
        case 15841: launch_split<15, 8, 4, 1, INV>(p, n_limbs, s); break;
        case 15850: launch_split<15, 8, 5, 0, INV>(p, n_limbs, s); break;
        case 15851: launch_split<15, 8, 5, 1, INV>(p, n_limbs, s); break;
        default: throw Error(VR_EINVAL, "ntt: no two-pass kernel for this split");
        }
        VR_CHECK_LAUNCH();
        return;
    }
    if (c.direct == 2) {
        // whole-limb kernel with the geometry fixed at compile time
        switch (p.log_n * 100 + c.div) {
        case 1316: launch_limb<13, 4, INV>(p, n_limbs, s); break;
        case 1332: launch_limb<13, 5, INV>(p, n_limbs, s); break;
        case 1416: launch_limb<14, 4, INV>(p, n_limbs, s); break;
        case 1432: launch_limb<14, 5, INV>(p, n_limbs, s); break;
        default: throw Error(VR_EINVAL, "ntt: no whole-limb kernel for this size");
        }
        VR_CHECK_LAUNCH();
        return;
    }
    u32 tile = 1u << (p.log_g + p.log_c);
    u32 threads = tile / c.div;
    if (threads < 64) threads = 64;
    if (threads > 1024) throw Error(VR_EINVAL, "ntt: tile too large");
    const bool direct = c.direct && p.log_c == 0 && p.log_g == p.log_n;
    if (direct && threads > 512) throw Error(VR_EINVAL, "ntt: whole-limb pass needs <= 512 threads");
    u32 blocks = n_limbs * ((1u << (p.log_n - p.log_g - p.log_c)));
    size_t shmem = (size_t)(tile + tile / 16) * sizeof(u64);
    if (p.max_r == 5) {
        // five-stage rounds: whole-limb passes with 32 words per thread only
        if (!direct || c.div != 32) throw Error(VR_EINVAL, "ntt: five-stage rounds need a direct pass");
        switch (threads) {
        case 256: launch_kernel<256, INV, true, true>(p, blocks, shmem, s); break;
        case 512: launch_kernel<512, INV, true, true>(p, blocks, shmem, s); break;
        default: throw Error(VR_EINVAL, "ntt: unsupported tile for five-stage rounds");
        }
        VR_CHECK_LAUNCH();
        return;
    }
    switch (threads) {
    case 64: direct ? launch_kernel<64, INV, true>(p, blocks, shmem, s) : launch_kernel<64, INV, false>(p, blocks, shmem, s); break;
    case 128: direct ? launch_kernel<128, INV, true>(p, blocks, shmem, s) : launch_kernel<128, INV, false>(p, blocks, shmem, s); break;
    case 256: direct ? launch_kernel<256, INV, true>(p, blocks, shmem, s) : launch_kernel<256, INV, false>(p, blocks, shmem, s); break;
    case 512: direct ? launch_kernel<512, INV, true>(p, blocks, shmem, s) : launch_kernel<512, INV, false>(p, blocks, shmem, s); break;
    case 1024: launch_kernel<1024, INV, false>(p, blocks, shmem, s); break;
    default: throw Error(VR_EINVAL, "ntt: unsupported tile");
    }
    VR_CHECK_LAUNCH();
}

// Limbs per launch pair of the compile-time two-pass kernels (0: all limbs in
// one launch per pass).  With chunks, pass 0 and pass 1 alternate chunk by
// chunk, so the intermediate pass 1 reads was written moments before and is
// still in the last-level cache.
u32 split_chunk(vr_context* ctx)
{
    std::lock_guard<std::mutex> g(ctx->mu);
    auto it = ctx->tuning.find("ntt_chunk");
    return it == ctx->tuning.end() ? kSplitChunkDefault : (u32)it->second;
}

template <bool INV>
void run_plan(vr_context* ctx, const LimbSet& ls, const std::vector<PassCfg>& passes, hipStream_t s)
{
    u32 n_limbs = ls.per_poly * ls.n_polys;
    NttPass p;
    p.ls = ls;
    p.mq = ctx->d_modq;
    p.tw = INV ? ctx->d_itw : ctx->d_tw;
    p.twf = INV ? ctx->d_itwf : ctx->d_twf;
    p.log_n = ctx->log_n;
    p.L = ctx->L;
    p.r0 = 0;
    size_t np = passes.size();
    // every limb's two passes touch only that limb's words (and shared
    // tables), so the limbs may run in chunks
    const u32 chunk = np == 2 && passes[0].direct == 3 ? split_chunk(ctx) : 0;
    const u32 step = chunk ? chunk : n_limbs;
    for (u32 r0 = 0; r0 < n_limbs; r0 += step) {
        p.r0 = r0;
        const u32 nc = std::min(step, n_limbs - r0);
        for (size_t i = 0; i < np; i++) {
            // forward runs the stage groups in order, inverse in reverse
            const PassCfg& c = INV ? passes[np - 1 - i] : passes[i];
            p.s0 = c.s0;
            p.log_g = c.log_g;
            p.log_c = c.log_c;
            p.first = (i == 0);
            p.last = (i == np - 1);
            p.max_r = c.max_r;
            launch_pass<INV>(p, c, nc, s);
        }
    }
}

// Times every candidate plan on 256-2048 scratch limbs of the Q chain (five runs
// each after a warm-up) and keeps the fastest; a later candidate replaces an
// earlier one only when it is more than 8 % faster, so that plans within the
// timing noise of each other do not flip from run to run.
template <bool INV>
std::vector<PassCfg> tune(vr_context* ctx, hipStream_t s)
{
    auto cands = candidates(ctx->log_n);
    if (cands.size() < 2) return cands.empty() ? default_plan(ctx->log_n) : cands[0];
    // several limbs per CU, as in a layer's launches, within 256 MiB
    const u32 want = std::max(256u, std::min(2048u, (u32)((256u << 20) / (8ull * ctx->n))));
    const u32 per = ctx->L + 1, polys = (want + per - 1) / per;
    const size_t words = (size_t)per * polys * ctx->n;
    void* buf = ctx->arena->alloc(words * sizeof(u64), s);
    if (!buf) return default_plan(ctx->log_n);
    VR_HIP(hipMemsetAsync(buf, 0, words * sizeof(u64), s));
    LimbSet ls = poly_limbs((u64*)buf, (u64*)buf, polys, per, (u64)per * ctx->n, (int)ctx->L);
    hipEvent_t a, b;
    VR_HIP(hipEventCreate(&a));
    VR_HIP(hipEventCreate(&b));
    float best = 1e30f;
    size_t pick = 0;
    for (size_t i = 0; i < cands.size(); i++) {
        run_plan<INV>(ctx, ls, cands[i], s);
        VR_HIP(hipEventRecord(a, s));
        for (int r = 0; r < 5; r++) run_plan<INV>(ctx, ls, cands[i], s);
        VR_HIP(hipEventRecord(b, s));
        VR_HIP(hipEventSynchronize(b));
        float ms = 0;
        VR_HIP(hipEventElapsedTime(&ms, a, b));
        if (ms < best * 0.92f) best = ms, pick = i;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    ctx->arena->release(buf, s);
    return cands[pick];
}

template <bool INV>
std::vector<PassCfg> plan_for(vr_context* ctx, hipStream_t s)
{
    int mode = 0;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->tuning.find("ntt");
        if (it != ctx->tuning.end()) mode = it->second;
        if (mode == 0 && !ctx->ntt_plan[INV].empty()) {
            std::vector<PassCfg> p;
            for (auto& c : ctx->ntt_plan[INV]) p.push_back({c[0], c[1], c[2], c[3], c[4], c[5]});
            return p;
        }
    }
    if (mode >= 2) {
        auto cands = candidates(ctx->log_n);
        if ((size_t)(mode - 2) >= cands.size()) throw Error(VR_EINVAL, "ntt: no such candidate plan");
        return cands[mode - 2];
    }
    if (mode == 1 || g_capture) return default_plan(ctx->log_n);
    std::vector<PassCfg> p = tune<INV>(ctx, s);
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->ntt_plan[INV].clear();
    for (auto& c : p) ctx->ntt_plan[INV].push_back({c.s0, c.log_g, c.log_c, c.direct, c.div, c.max_r});
    return p;
}

// Runs the transform; a forward epilogue is applied when the plan is one
// whole-limb pass or ends with a compile-time two-pass kernel, else dropped
// (the transform is stored) and false returned.
template <bool INV>
bool run(vr_context* ctx, const LimbSet& ls, hipStream_t s)
{
    u32 n_limbs = ls.per_poly * ls.n_polys;
    std::vector<PassCfg> passes = plan_for<INV>(ctx, s);
    const bool fuse = !INV && ls.epi.a &&
                      ((passes.size() == 1 && passes[0].direct == 2) ||
                       (passes.size() == 2 && passes[1].direct == 3));
    if (n_limbs == 0) return fuse;
    ProfScope prof(ctx, kProfNtt, s, n_limbs);
    if (fuse || !ls.epi.a) {
        run_plan<INV>(ctx, ls, passes, s);
    } else {
        LimbSet plain = ls;
        plain.epi = NttEpilogue();
        run_plan<INV>(ctx, plain, passes, s);
    }
    return fuse;
}

}  // namespace

bool ntt_forward(vr_context* ctx, const LimbSet& ls, hipStream_t s) { return run<false>(ctx, ls, s); }
void ntt_inverse(vr_context* ctx, const LimbSet& ls, hipStream_t s) { (void)run<true>(ctx, ls, s); }

}  // namespace vr
