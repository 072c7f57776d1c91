// Element-wise RNS kernels (modular Hadamard products and friends), rescale
// helpers and the evaluation-domain Galois automorphism.
//
// These are HBM-streaming kernels: every thread owns two consecutive
// coefficients of one limb (one 16-byte load per operand), a 256-thread block
// covers 512 coefficients, so with N >= 512 a block never straddles limbs and
// the modulus constants are wave-uniform.
#include "vr_ops.h"

namespace vr {

namespace {

constexpr int kThreads = 256;

inline dim3 grid_for(size_t elems)
{
    size_t pairs = (elems + 1) / 2;
    return dim3((unsigned)((pairs + kThreads - 1) / kThreads));
}


__global__ void k_addsub(u64* out, const u64* a, const u64* b, size_t elems, u32 log_n, u32 nl,
                         const ModQ* mq, int sub)
{
    size_t e = 2 * ((size_t)blockIdx.x * kThreads + threadIdx.x);
    if (e >= elems) return;
    u32 l = (u32)((e >> log_n) % nl);
    u64 q = mq[l].q;
    ulonglong2 x = *(const ulonglong2*)(a + e);
    ulonglong2 y = *(const ulonglong2*)(b + e);
    ulonglong2 r;
    if (sub) {
        r.x = sub_mod(x.x, y.x, q);
        r.y = sub_mod(x.y, y.y, q);
    } else {
        r.x = add_mod(x.x, y.x, q);
        r.y = add_mod(x.y, y.y, q);
    }
    *(ulonglong2*)(out + e) = r;
}

__global__ void k_mul_scalar(u64* out, const u64* a, size_t elems, u32 log_n, u32 nl,
                             const ModQ* mq, LimbConsts c)
{
    size_t e = 2 * ((size_t)blockIdx.x * kThreads + threadIdx.x);
    if (e >= elems) return;
    u32 l = (u32)((e >> log_n) % nl);
    u64 q = mq[l].q, w = c.c[l], ws = c.cs[l];
    ulonglong2 x = *(const ulonglong2*)(a + e);
    ulonglong2 r;
    r.x = shoup(x.x, w, ws, q);
    r.y = shoup(x.y, w, ws, q);
    *(ulonglong2*)(out + e) = r;
}

__global__ void k_add_scalar(u64* out, const u64* a, size_t elems, u32 log_n, const ModQ* mq,
                             LimbConsts c)
{
    size_t e = 2 * ((size_t)blockIdx.x * kThreads + threadIdx.x);
    if (e >= elems) return;
    u32 l = (u32)(e >> log_n);
    u64 q = mq[l].q, w = c.c[l];
    ulonglong2 x = *(const ulonglong2*)(a + e);
    ulonglong2 r;
    r.x = add_mod(x.x, w, q);
    r.y = add_mod(x.y, w, q);
    *(ulonglong2*)(out + e) = r;
}

__global__ void k_mul_plain(u64* out, const u64* a, const u64* pt, size_t elems, u32 log_n, u32 nl,
                            const ModQ* mq)
{
    size_t e = 2 * ((size_t)blockIdx.x * kThreads + threadIdx.x);
    if (e >= elems) return;
    size_t r = e >> log_n;
    u32 l = (u32)(r % nl);
    const ModQ m = mq[l];
    size_t pe = ((size_t)l << log_n) + (e & ((1u << log_n) - 1));
    ulonglong2 x = *(const ulonglong2*)(a + e);
    ulonglong2 y = *(const ulonglong2*)(pt + pe);
    ulonglong2 o;
    o.x = mul_mod(x.x, y.x, m);
    o.y = mul_mod(x.y, y.y, m);
    *(ulonglong2*)(out + e) = o;
}

__global__ void k_tensor(u64* out, const u64* a, const u64* b, size_t poly_elems, u32 log_n,
                         const ModQ* mq)
{
    size_t e = 2 * ((size_t)blockIdx.x * kThreads + threadIdx.x);
    if (e >= poly_elems) return;
    u32 l = (u32)(e >> log_n);
    const ModQ m = mq[l];
    ulonglong2 a0 = *(const ulonglong2*)(a + e);
    ulonglong2 a1 = *(const ulonglong2*)(a + poly_elems + e);
    ulonglong2 b0 = *(const ulonglong2*)(b + e);
    ulonglong2 b1 = *(const ulonglong2*)(b + poly_elems + e);
    ulonglong2 d0, d1, d2;
    d0.x = mul_mod(a0.x, b0.x, m);
    d0.y = mul_mod(a0.y, b0.y, m);
    d1.x = add_mod(mul_mod(a0.x, b1.x, m), mul_mod(a1.x, b0.x, m), m.q);
    d1.y = add_mod(mul_mod(a0.y, b1.y, m), mul_mod(a1.y, b0.y, m), m.q);
    d2.x = mul_mod(a1.x, b1.x, m);
    d2.y = mul_mod(a1.y, b1.y, m);
    *(ulonglong2*)(out + e) = d0;
    *(ulonglong2*)(out + poly_elems + e) = d1;
    *(ulonglong2*)(out + 2 * poly_elems + e) = d2;
}

__global__ void k_automorphism(u64* out, const u64* a, u32 n_polys, u32 nl, u64 poly_stride,
                               u32 log_n, u32 g)
{
    size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
    size_t n = (size_t)1 << log_n;
    size_t total = (size_t)n_polys * nl * n;
    if (idx >= total) return;
    size_t r = idx >> log_n;
    u32 i = (u32)(idx & (n - 1));
    size_t p = r / nl, l = r - p * nl;
    size_t base = p * poly_stride + l * n;
    out[base + i] = a[base + galois_src(i, g, log_n)];
}

// r[k][i][t] = [centred coef[k][t]]_{q_i} for i < level, coef modulo q_level
__global__ void k_rescale_spread(u64* r, const u64* coef, u32 n_polys, u32 level, u32 log_n,
                                 const ModQ* mq)
{
    size_t e = 2 * ((size_t)blockIdx.x * kThreads + threadIdx.x);
    size_t n = (size_t)1 << log_n;
    size_t total = (size_t)n_polys * level * n;
    if (e >= total) return;
    size_t row = e >> log_n;
    u32 k = (u32)(row / level), i = (u32)(row % level);
    size_t t = e & (n - 1);
    u64 ql = mq[level].q;
    const ModQ mi = mq[i];
    ulonglong2 x = *(const ulonglong2*)(coef + (size_t)k * n + t);
    ulonglong2 o;
    // centred value c - q_l when c > q_l / 2: [c - q_l]_{q_i} = -[q_l - c]_{q_i}
    o.x = x.x > (ql >> 1) ? neg_mod(red64(ql - x.x, mi), mi.q) : red64(x.x, mi);
    o.y = x.y > (ql >> 1) ? neg_mod(red64(ql - x.y, mi), mi.q) : red64(x.y, mi);
    *(ulonglong2*)(r + e) = o;
}

__global__ void k_rescale_finish(u64* out, const u64* c, const u64* r, u32 n_polys, u32 level,
                                 u32 log_n, const ModQ* mq, LimbConsts qinv)
{
    size_t e = 2 * ((size_t)blockIdx.x * kThreads + threadIdx.x);
    size_t n = (size_t)1 << log_n;
    size_t total = (size_t)n_polys * level * n;
    if (e >= total) return;
    size_t row = e >> log_n;
    u32 k = (u32)(row / level), i = (u32)(row % level);
    size_t t = e & (n - 1);
    u64 q = mq[i].q;
    ulonglong2 x = *(const ulonglong2*)(c + ((size_t)k * (level + 1) + i) * n + t);
    ulonglong2 y = *(const ulonglong2*)(r + e);
    ulonglong2 o;
    o.x = shoup(x.x + q - y.x, qinv.c[i], qinv.cs[i], q);
    o.y = shoup(x.y + q - y.y, qinv.c[i], qinv.cs[i], q);
    *(ulonglong2*)(out + e) = o;
}

__global__ void k_int_to_limbs(u64* out, const i64* x, u32 n_mods, u32 log_n, const ModQ* mq,
                               LimbConsts mods)
{
    size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
    size_t n = (size_t)1 << log_n;
    if (idx >= (size_t)n_mods * n) return;
    u32 l = (u32)(idx >> log_n);
    const ModQ m = mq[mods.c[l]];
    i64 v = x[idx & (n - 1)];
    out[idx] = v >= 0 ? red64((u64)v, m) : neg_mod(red64((u64)(-(v + 1)) + 1, m), m.q);
}

// rows of `width` words: dst + r * dst_stride <- src + r * src_stride
__global__ void k_copy_rows(u64* dst, u64 dst_stride, const u64* src, u64 src_stride, u64 width,
                            u32 rows)
{
    size_t idx = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= width * rows) return;
    size_t r = idx / width, c = idx - r * width;
    dst[r * dst_stride + c] = src[r * src_stride + c];
}

}  // namespace

void launch_copy_rows(u64* dst, u64 dst_stride, const u64* src, u64 src_stride, u64 width, u32 rows,
                      hipStream_t s)
{
    size_t total = (size_t)width * rows;
    if (total == 0) return;
    hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)((total + kThreads - 1) / kThreads)), dim3(kThreads),
                       0, s, dst, dst_stride, src, src_stride, width, rows);
    VR_CHECK_LAUNCH();
}

void launch_addsub(vr_context* ctx, u64* out, const u64* a, const u64* b, u32 n_polys, u32 nl,
                   bool sub, hipStream_t s)
{
    size_t elems = (size_t)n_polys * nl * ctx->n;
    hipLaunchKernelGGL(k_addsub, grid_for(elems), dim3(kThreads), 0, s, out, a, b, elems,
                       ctx->log_n, nl, ctx->d_modq, sub ? 1 : 0);
    VR_CHECK_LAUNCH();
}

void launch_mul_scalar(vr_context* ctx, u64* out, const u64* a, u32 n_polys, u32 nl,
                       const LimbConsts& c, hipStream_t s)
{
    size_t elems = (size_t)n_polys * nl * ctx->n;
    hipLaunchKernelGGL(k_mul_scalar, grid_for(elems), dim3(kThreads), 0, s, out, a, elems,
                       ctx->log_n, nl, ctx->d_modq, c);
    VR_CHECK_LAUNCH();
}

void launch_add_scalar(vr_context* ctx, u64* out, const u64* a, u32 nl, const LimbConsts& c,
                       hipStream_t s)
{
    size_t elems = (size_t)nl * ctx->n;
    hipLaunchKernelGGL(k_add_scalar, grid_for(elems), dim3(kThreads), 0, s, out, a, elems,
                       ctx->log_n, ctx->d_modq, c);
    VR_CHECK_LAUNCH();
}

void launch_mul_plain(vr_context* ctx, u64* out, const u64* a, const u64* pt, u32 n_polys, u32 nl,
                      hipStream_t s)
{
    size_t elems = (size_t)n_polys * nl * ctx->n;
    hipLaunchKernelGGL(k_mul_plain, grid_for(elems), dim3(kThreads), 0, s, out, a, pt, elems,
                       ctx->log_n, nl, ctx->d_modq);
    VR_CHECK_LAUNCH();
}

void launch_tensor(vr_context* ctx, u64* out, const u64* a, const u64* b, u32 nl, hipStream_t s)
{
    size_t elems = (size_t)nl * ctx->n;
    hipLaunchKernelGGL(k_tensor, grid_for(elems), dim3(kThreads), 0, s, out, a, b, elems,
                       ctx->log_n, ctx->d_modq);
    VR_CHECK_LAUNCH();
}

void launch_automorphism(vr_context* ctx, u64* out, const u64* a, u32 n_polys, u32 nl,
                         u64 poly_stride, u32 g, hipStream_t s)
{
    size_t total = (size_t)n_polys * nl * ctx->n;
    dim3 grid((unsigned)((total + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(k_automorphism, grid, dim3(kThreads), 0, s, out, a, n_polys, nl,
                       poly_stride, ctx->log_n, g);
    VR_CHECK_LAUNCH();
}

void launch_rescale_spread(vr_context* ctx, u64* r, const u64* coef, u32 n_polys, u32 level,
                           hipStream_t s)
{
    size_t elems = (size_t)n_polys * level * ctx->n;
    hipLaunchKernelGGL(k_rescale_spread, grid_for(elems), dim3(kThreads), 0, s, r, coef, n_polys,
                       level, ctx->log_n, ctx->d_modq);
    VR_CHECK_LAUNCH();
}

void launch_rescale_finish(vr_context* ctx, u64* out, const u64* c, const u64* r, u32 n_polys,
                           u32 level, hipStream_t s)
{
    LimbConsts qinv;
    u64 ql = ctx->mod[level];
    for (u32 i = 0; i < level; i++) {
        u64 q = ctx->mod[i];
        // q_l^-1 mod q_i by Fermat
        u64 base = ql % q, e = q - 2, acc = 1;
        while (e) {
            if (e & 1) acc = (u64)((u128)acc * base % q);
            base = (u64)((u128)base * base % q);
            e >>= 1;
        }
        qinv.c[i] = acc;
        qinv.cs[i] = shoup_companion(acc, q);
    }
    size_t elems = (size_t)n_polys * level * ctx->n;
    hipLaunchKernelGGL(k_rescale_finish, grid_for(elems), dim3(kThreads), 0, s, out, c, r, n_polys,
                       level, ctx->log_n, ctx->d_modq, qinv);
    VR_CHECK_LAUNCH();
}

void launch_int_to_limbs(vr_context* ctx, u64* out, const i64* x, const u32* mods_host, u32 n_mods,
                         hipStream_t s)
{
    LimbConsts mods;
    for (u32 i = 0; i < n_mods; i++) mods.c[i] = mods_host[i];
    size_t total = (size_t)n_mods * ctx->n;
    dim3 grid((unsigned)((total + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(k_int_to_limbs, grid, dim3(kThreads), 0, s, out, x, n_mods, ctx->log_n,
                       ctx->d_modq, mods);
    VR_CHECK_LAUNCH();
}

}  // namespace vr
