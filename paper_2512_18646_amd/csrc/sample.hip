// Randomness and the key-generation / encryption / decryption combiners.
//
// Stream: ChaCha20 (RFC 8439) keyed by the 256-bit seed (32 little-endian
// bytes), nonce = purpose (u32) || object id (u64), block counter
// from 0; 64-bit word w is bytes 8w..8w+7 of the keystream.  Every sample sits
// at a fixed word position, so one GPU thread computes one 64-byte block and
// emits the samples it holds, with no sequential dependence:
//   ternary   word t:                      floor(3 w / 2^64) - 1
//   gaussian  word t:                      sign bit 63, |x| = min{k : low63 < T[k]}
//   uniform   words 2(limb N + t), +1:     floor(W q / 2^128), W = hi:lo
#include "cdt_table.h"
#include "vr_ops.h"

namespace vr {

namespace {

constexpr int kThreads = 256;

__constant__ u64 c_cdt[20];

__device__ __forceinline__ u32 rotl(u32 x, int n) { return (x << n) | (x >> (32 - n)); }

#define VR_QR(a, b, c, d)                 \
    a += b; d ^= a; d = rotl(d, 16);      \
    c += d; b ^= c; b = rotl(b, 12);      \
    a += b; d ^= a; d = rotl(d, 8);       \
    c += d; b ^= c; b = rotl(b, 7);

// 16 output words of block `ctr` for (seed, purpose, obj)
__device__ void chacha_block(const Seed256& seed, u32 purpose, u64 obj, u32 ctr, u32 out[16])
{
    u32 x[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u,
                 (u32)seed.w[0], (u32)(seed.w[0] >> 32), (u32)seed.w[1], (u32)(seed.w[1] >> 32),
                 (u32)seed.w[2], (u32)(seed.w[2] >> 32), (u32)seed.w[3], (u32)(seed.w[3] >> 32),
                 ctr, purpose, (u32)obj, (u32)(obj >> 32)};
    u32 s[16];
#pragma unroll
    for (int i = 0; i < 16; i++) s[i] = x[i];
#pragma unroll
    for (int r = 0; r < 10; r++) {
        VR_QR(s[0], s[4], s[8], s[12]);
        VR_QR(s[1], s[5], s[9], s[13]);
        VR_QR(s[2], s[6], s[10], s[14]);
        VR_QR(s[3], s[7], s[11], s[15]);
        VR_QR(s[0], s[5], s[10], s[15]);
        VR_QR(s[1], s[6], s[11], s[12]);
        VR_QR(s[2], s[7], s[8], s[13]);
        VR_QR(s[3], s[4], s[9], s[14]);
    }
#pragma unroll
    for (int i = 0; i < 16; i++) out[i] = s[i] + x[i];
}

__global__ void k_sample_small(i64* out, Seed256 seed, u32 purpose, u64 obj, u32 n, int gauss)
{
    u32 b = blockIdx.x * kThreads + threadIdx.x;
    if (8 * b >= n) return;
    u32 blk[16];
    chacha_block(seed, purpose, obj, b, blk);
#pragma unroll
    for (int j = 0; j < 8; j++) {
        u64 w = (u64)blk[2 * j] | ((u64)blk[2 * j + 1] << 32);
        i64 v;
        if (!gauss) {
            v = (i64)mulhi64(w, 3) - 1;
        } else {
            u64 r = w & 0x7fffffffffffffffull;
            i64 k = 0;
#pragma unroll
            for (int i = 0; i < 19; i++) k += r >= c_cdt[i] ? 1 : 0;
            v = ((w >> 63) && k) ? -k : k;
        }
        if (8 * b + j < n) out[8 * b + j] = v;
    }
}

struct UniArgs {
    Seed256 seed;
    u64 obj;
    u32 purpose, log_n, n_limbs;
    u32 limb_index[kMaxMod];
    u32 mods[kMaxMod];
};
VR_KERNEL_ARG(UniArgs);

__global__ void k_sample_uniform(u64* out, UniArgs a, const ModQ* mq)
{
    const u32 n = 1u << a.log_n;
    u32 tid = blockIdx.x * kThreads + threadIdx.x;   // 4 coefficients per thread
    u32 per_limb = n / 4;
    if (tid >= per_limb * a.n_limbs) return;
    u32 r = tid / per_limb;
    u32 t0 = (tid - r * per_limb) * 4;
    u64 q = mq[a.mods[r]].q;
    // word index of coefficient t0: 2 (limb N + t0), a multiple of 8
    u64 w0 = 2 * ((u64)a.limb_index[r] * n + t0);
    u32 blk[16];
    chacha_block(a.seed, a.purpose, a.obj, (u32)(w0 / 8), blk);
#pragma unroll
    for (int j = 0; j < 4; j++) {
        u64 lo = (u64)blk[4 * j] | ((u64)blk[4 * j + 1] << 32);
        u64 hi = (u64)blk[4 * j + 2] | ((u64)blk[4 * j + 3] << 32);
        // floor((hi 2^64 + lo) q / 2^128) = (hi q + floor(lo q / 2^64)) >> 64
        u64 mid = mulhi64(lo, q);
        u64 plo = hi * q;
        u64 phi = mulhi64(hi, q);
        u64 s = plo + mid;
        phi += s < plo ? 1 : 0;
        out[(size_t)r * n + t0 + j] = phi;
    }
}

// limb l of b, a, e is modulus index l
__global__ void k_key_combine(u64* b, const u64* a, const u64* e, const u64* s_all,
                              const u64* sp_all, u32 n, u32 log_n, const ModQ* mq, u32 dlo, u32 dhi)
{
    size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
    size_t N = (size_t)1 << log_n;
    if (idx >= (size_t)n * N) return;
    u32 l = (u32)(idx >> log_n);
    const ModQ m = mq[l];
    u64 as = mul_mod(a[idx], s_all[idx], m);
    u64 v = sub_mod(e[idx], as, m.q);
    if (l >= dlo && l < dhi) v = add_mod(v, shoup(sp_all[idx], m.pmod, m.pmod_s, m.q), m.q);
    b[idx] = v;
}

__global__ void k_encrypt_combine(u64* ct, const u64* v, const u64* e0, const u64* e1,
                                  const u64* pk, const u64* msg, u32 nl, u32 pk_nl, u32 log_n,
                                  const ModQ* mq)
{
    size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
    size_t N = (size_t)1 << log_n;
    if (idx >= (size_t)nl * N) return;
    u32 l = (u32)(idx >> log_n);
    const ModQ m = mq[l];
    u64 vv = v[idx];
    u64 c0 = add_mod(add_mod(mul_mod(vv, pk[idx], m), e0[idx], m.q), msg[idx], m.q);
    u64 c1 = add_mod(mul_mod(vv, pk[(size_t)pk_nl * N + idx], m), e1[idx], m.q);
    ct[idx] = c0;
    ct[(size_t)nl * N + idx] = c1;
}

__global__ void k_decrypt_combine(u64* msg, const u64* ct, u32 ncomp, const u64* s_all, u32 nl,
                                  u32 log_n, const ModQ* mq)
{
    size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
    size_t N = (size_t)1 << log_n;
    if (idx >= (size_t)nl * N) return;
    u32 l = (u32)(idx >> log_n);
    const ModQ m = mq[l];
    u64 s = s_all[idx];
    u64 acc = ct[idx];
    u64 sp = s;
    for (u32 k = 1; k < ncomp; k++) {
        acc = add_mod(acc, mul_mod(ct[(size_t)k * nl * N + idx], sp, m), m.q);
        sp = mul_mod(sp, s, m);
    }
    msg[idx] = acc;
}

bool g_cdt_loaded = false;

}  // namespace

void upload_cdt(hipStream_t s)
{
    if (g_cdt_loaded) return;
    VR_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_cdt), kGaussCdt, sizeof(kGaussCdt)));
    g_cdt_loaded = true;
}

void launch_sample_ternary(vr_context* ctx, i64* out, const Seed256& seed, u32 purpose, u64 obj, hipStream_t s)
{
    u32 blocks = (ctx->n / 8 + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_sample_small, dim3(blocks), dim3(kThreads), 0, s, out, seed, purpose, obj,
                       ctx->n, 0);
    VR_CHECK_LAUNCH();
}

void launch_sample_gauss(vr_context* ctx, i64* out, const Seed256& seed, u32 purpose, u64 obj, hipStream_t s)
{
    upload_cdt(s);
    u32 blocks = (ctx->n / 8 + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_sample_small, dim3(blocks), dim3(kThreads), 0, s, out, seed, purpose, obj,
                       ctx->n, 1);
    VR_CHECK_LAUNCH();
}

void launch_sample_uniform(vr_context* ctx, u64* out, const Seed256& seed, u32 purpose, u64 obj,
                           const u32* limb_index_host, const u32* mods_host, u32 n, hipStream_t s)
{
    UniArgs a;
    a.seed = seed;
    a.obj = obj;
    a.purpose = purpose;
    a.log_n = ctx->log_n;
    a.n_limbs = n;
    for (u32 i = 0; i < n; i++) {
        a.limb_index[i] = limb_index_host[i];
        a.mods[i] = mods_host[i];
    }
    u32 total = n * (ctx->n / 4);
    hipLaunchKernelGGL(k_sample_uniform, dim3((total + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       s, out, a, ctx->d_modq);
    VR_CHECK_LAUNCH();
}

void launch_key_combine(vr_context* ctx, u64* b, const u64* a, const u64* e, const u64* s_all,
                        const u64* sp_all, u32 n, u32 dlo, u32 dhi, hipStream_t st)
{
    size_t total = (size_t)n * ctx->n;
    hipLaunchKernelGGL(k_key_combine, dim3((unsigned)((total + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, st, b, a, e, s_all, sp_all, n, ctx->log_n, ctx->d_modq,
                       dlo, dhi);
    VR_CHECK_LAUNCH();
}

void launch_encrypt_combine(vr_context* ctx, u64* ct, const u64* v, const u64* e0, const u64* e1,
                            const u64* pk, const u64* m, u32 nl, hipStream_t s)
{
    size_t total = (size_t)nl * ctx->n;
    hipLaunchKernelGGL(k_encrypt_combine, dim3((unsigned)((total + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, ct, v, e0, e1, pk, m, nl, ctx->L + 1, ctx->log_n,
                       ctx->d_modq);
    VR_CHECK_LAUNCH();
}

void launch_decrypt_combine(vr_context* ctx, u64* m, const u64* ct, u32 ncomp, const u64* s_all,
                            u32 nl, hipStream_t s)
{
    size_t total = (size_t)nl * ctx->n;
    hipLaunchKernelGGL(k_decrypt_combine, dim3((unsigned)((total + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, m, ct, ncomp, s_all, nl, ctx->log_n, ctx->d_modq);
    VR_CHECK_LAUNCH();
}

}  // namespace vr
