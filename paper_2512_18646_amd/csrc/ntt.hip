// Negacyclic NTT / inverse NTT on gfx950.
//
// Transform: out[i] = sum_t a_t psi^((2 brev(i) + 1) t) mod q (bit-reversed
// evaluation order), computed as the radix-2 Cooley-Tukey network with merged
// psi twiddles; the inverse is the Gentleman-Sande network with inverse
// twiddles followed by N^-1.
//
// A limb is N uint64 (64 KiB at N = 2^13, 128 KiB at 2^14, 512 KiB at 2^16).
// Up to 2^14 one workgroup holds a whole limb in LDS (160 KiB per CU) and runs
// every stage there: one HBM read and one write per limb.  At 2^15 and 2^16 the
// limb does not fit, so the stages split in two passes over groups of
// 2^log_g elements: the first pass works on strided groups (the high index bits
// vary) with 16-32 consecutive groups per workgroup so every row read is a
// coalesced 128-256 byte segment; the second pass on contiguous blocks.
// Butterflies use Shoup products with precomputed twiddle companions and lazy
// reduction (forward values in [0, 4q), inverse in [0, 2q); Harvey 2014),
// reduced to [0, q) only when the last pass stores.
#include "vr_core.h"

namespace vr {

struct NttPass {
    LimbSet ls;
    const ModQ* mq;
    const u64* tw;      // [nmod][N]
    const u64* tw_s;
    u32 log_n, L;
    u32 s0, log_g, log_c;
    u32 first, last;
};

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
    size_t off = (size_t)poly * ls.poly_stride + (size_t)slot * n;
    *in = ls.in + off;
    *out = ls.out_dense ? ls.out + (size_t)r * n : ls.out + off;
}

template <int THREADS, bool INV>
__global__ __launch_bounds__(THREADS) void k_ntt_pass(NttPass p)
{
    extern __shared__ u64 lds[];
    const u32 n = 1u << p.log_n;
    const u32 G = 1u << p.log_g;
    const u32 C = 1u << p.log_c;
    const u32 tile = G << p.log_c;
    const u32 lo_bits = p.log_n - p.s0 - p.log_g;
    const u32 blocks_per_limb = (n >> p.log_g) >> p.log_c;
    const u32 r = blockIdx.x / blocks_per_limb;
    const u32 g0 = (blockIdx.x - r * blocks_per_limb) << p.log_c;

    const u64* src;
    u64* dst;
    u32 mod;
    limb_addr(p.ls, r, n, p.L, &src, &dst, &mod);
    if (!p.first) src = dst;
    const ModQ m = p.mq[mod];
    const u64 q = m.q, q2 = 2 * m.q;
    const u64* tw = p.tw + (size_t)mod * n;
    const u64* tws = p.tw_s + (size_t)mod * n;

    // coalesced load: consecutive threads take consecutive addresses
    const bool strided = lo_bits > 0;
    for (u32 e = threadIdx.x; e < tile; e += THREADS) {
        u32 c, v;
        if (strided) { v = e >> p.log_c; c = e & (C - 1); }
        else { c = e >> p.log_g; v = e & (G - 1); }
        u32 g = g0 + c;
        u32 H = g >> lo_bits, Lo = g & ((1u << lo_bits) - 1);
        size_t idx = ((size_t)H << (p.log_n - p.s0)) + ((size_t)v << lo_bits) + Lo;
        lds[c * G + v] = src[idx];
    }
    __syncthreads();

    const u32 half = tile >> 1;
    if (!INV) {
        for (u32 sg = 0; sg < p.log_g; sg++) {
            const u32 t = G >> (sg + 1);
            const u32 s = p.s0 + sg;
            for (u32 b = threadIdx.x; b < half; b += THREADS) {
                u32 c = b >> (p.log_g - 1);
                u32 k = b & ((G >> 1) - 1);
                u32 v1 = ((k & ~(t - 1)) << 1) | (k & (t - 1));
                u32 H = (g0 + c) >> lo_bits;
                u32 ti = (1u << s) + (H << sg) + (v1 >> (p.log_g - sg));
                u64 w = tw[ti], ws = tws[ti];
                u64 X = lds[c * G + v1];
                u64 Y = lds[c * G + v1 + t];
                X = X >= q2 ? X - q2 : X;
                u64 T = shoup_lazy(Y, w, ws, q);
                lds[c * G + v1] = X + T;
                lds[c * G + v1 + t] = X + q2 - T;
            }
            __syncthreads();
        }
    } else {
        for (int sg = (int)p.log_g - 1; sg >= 0; sg--) {
            const u32 t = G >> (sg + 1);
            const u32 s = p.s0 + sg;
            for (u32 b = threadIdx.x; b < half; b += THREADS) {
                u32 c = b >> (p.log_g - 1);
                u32 k = b & ((G >> 1) - 1);
                u32 v1 = ((k & ~(t - 1)) << 1) | (k & (t - 1));
                u32 H = (g0 + c) >> lo_bits;
                u32 ti = (1u << s) + (H << sg) + (v1 >> (p.log_g - sg));
                u64 w = tw[ti], ws = tws[ti];
                u64 X = lds[c * G + v1];
                u64 Y = lds[c * G + v1 + t];
                u64 S = X + Y;
                S = S >= q2 ? S - q2 : S;
                lds[c * G + v1] = S;
                lds[c * G + v1 + t] = shoup_lazy(X + q2 - Y, w, ws, q);
            }
            __syncthreads();
        }
    }

    for (u32 e = threadIdx.x; e < tile; e += THREADS) {
        u32 c, v;
        if (strided) { v = e >> p.log_c; c = e & (C - 1); }
        else { c = e >> p.log_g; v = e & (G - 1); }
        u32 g = g0 + c;
        u32 H = g >> lo_bits, Lo = g & ((1u << lo_bits) - 1);
        size_t idx = ((size_t)H << (p.log_n - p.s0)) + ((size_t)v << lo_bits) + Lo;
        u64 x = lds[c * G + v];
        if (p.last) {
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

namespace {

struct PassCfg {
    u32 s0, log_g, log_c;
};

std::vector<PassCfg> plan(u32 log_n)
{
    if (log_n <= 14) return {{0, log_n, 0}};
    if (log_n == 15) return {{0, 7, 5}, {7, 8, 4}};
    return {{0, 8, 4}, {8, 8, 4}};   // 2^16
}

template <bool INV>
void launch_pass(const NttPass& p, u32 n_limbs, hipStream_t s)
{
    u32 tile = 1u << (p.log_g + p.log_c);
    u32 threads = tile / 16;
    if (threads < 64) threads = 64;
    if (threads > 1024) threads = 1024;
    u32 blocks = n_limbs * ((1u << (p.log_n - p.log_g - p.log_c)));
    size_t shmem = (size_t)tile * sizeof(u64);
    switch (threads) {
#define VR_NTT_CASE(T)                                                                          \
    case T: {                                                                                   \
        static bool attr = false;                                                               \
        if (!attr) {                                                                            \
            VR_HIP(hipFuncSetAttribute((const void*)k_ntt_pass<T, INV>,                         \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024)); \
            attr = true;                                                                        \
        }                                                                                       \
        hipLaunchKernelGGL((k_ntt_pass<T, INV>), dim3(blocks), dim3(T), shmem, s, p);           \
        break;                                                                                  \
    }
        VR_NTT_CASE(64)
        VR_NTT_CASE(128)
        VR_NTT_CASE(256)
        VR_NTT_CASE(512)
        VR_NTT_CASE(1024)
#undef VR_NTT_CASE
    default:
        throw Error(VR_EINVAL, "ntt: unsupported tile");
    }
    VR_CHECK_LAUNCH();
}

template <bool INV>
void run(vr_context* ctx, const LimbSet& ls, hipStream_t s)
{
    u32 n_limbs = ls.per_poly * ls.n_polys;
    if (n_limbs == 0) return;
    ProfScope prof(ctx, kProfNtt, s, n_limbs);
    auto passes = plan(ctx->log_n);
    NttPass p;
    p.ls = ls;
    p.mq = ctx->d_modq;
    p.tw = INV ? ctx->d_itw : ctx->d_tw;
    p.tw_s = INV ? ctx->d_itw_s : ctx->d_tw_s;
    p.log_n = ctx->log_n;
    p.L = ctx->L;
    size_t np = passes.size();
    for (size_t i = 0; i < np; i++) {
        // forward runs the stage groups in order, inverse in reverse
        const PassCfg& c = INV ? passes[np - 1 - i] : passes[i];
        p.s0 = c.s0;
        p.log_g = c.log_g;
        p.log_c = c.log_c;
        p.first = (i == 0);
        p.last = (i == np - 1);
        launch_pass<INV>(p, n_limbs, s);
    }
}

}  // namespace

void ntt_forward(vr_context* ctx, const LimbSet& ls, hipStream_t s) { run<false>(ctx, ls, s); }
void ntt_inverse(vr_context* ctx, const LimbSet& ls, hipStream_t s) { run<true>(ctx, ls, s); }

}  // namespace vr
