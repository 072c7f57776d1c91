// The HE evaluator on handles: client calls (keygen, encode, encrypt,
// decrypt) and server calls (add, cMul, Mul, rescale, rotate), composed from
// the kernels in ops/ntt/keyswitch/sample/fft.
#include <cmath>

#include "eval.h"

namespace vr {

// ------------------------------------------------------------------ memory

DevBuf::~DevBuf()
{
    if (!ptr) return;
    if (cap)
        cap->give_back(ptr);
    else if (free_fn)
        free_fn(ptr, (void*)stream, free_user);
    else if (arena)
        arena->release(ptr, stream);
}

thread_local std::shared_ptr<CaptureKeep> g_capture;

void* CaptureKeep::take(size_t bytes)
{
    const size_t want = DeviceArena::round_size(bytes);
    std::lock_guard<std::mutex> g(mu);
    auto it = free.lower_bound(want);
    if (it != free.end() && it->first <= want + want / 4 + 4096) {
        void* p = it->second;
        free.erase(it);
        return p;
    }
    void* p = arena->alloc_fresh(bytes);
    if (p) size[p] = want;
    return p;
}

void CaptureKeep::give_back(void* p)
{
    std::lock_guard<std::mutex> g(mu);
    free.insert({size.at(p), p});
}

CaptureKeep::~CaptureKeep()
{
    // the graph is gone (its owner synchronised the device); later frees
    // follow the context's stream
    for (auto& kv : size) arena->release(kv.first, release_stream);
}

BufPtr dev_alloc(vr_context* ctx, size_t bytes, hipStream_t s)
{
    auto b = std::make_shared<DevBuf>();
    b->bytes = bytes;
    b->stream = s;
    if (bytes == 0) return b;
    if (g_capture) {
        b->ptr = g_capture->take(bytes);
        if (!b->ptr) throw Error(VR_ENOMEM, "device allocation failed");
        b->cap = g_capture;
    } else if (ctx->alloc_fn) {
        b->ptr = ctx->alloc_fn(bytes, (void*)s, ctx->alloc_user);
        if (!b->ptr) throw Error(VR_ENOMEM, "allocator hook returned NULL");
        b->free_fn = ctx->free_fn;
        b->free_user = ctx->alloc_user;
    } else {
        b->ptr = ctx->arena->alloc(bytes, s);
        if (!b->ptr) {
            size_t reserved = 0, in_use = 0;
            ctx->arena->usage(&reserved, &in_use);
            throw Error(VR_ENOMEM, "device allocation of " + std::to_string(bytes >> 20) + " MiB failed (" +
                                       std::to_string(in_use >> 20) + " MiB in use, " +
                                       std::to_string(reserved >> 20) + " MiB reserved)");
        }
        b->arena = ctx->arena;
    }
    return b;
}

vr_ciphertext* new_ct(vr_context* ctx, u32 ncomp, u32 level, double scale, hipStream_t s)
{
    auto* ct = new vr_ciphertext;
    ct->ctx = ctx;
    ct->ncomp = ncomp;
    ct->level = level;
    ct->scale = scale;
    try {
        ct->buf = dev_alloc(ctx, (size_t)ncomp * (level + 1) * ctx->n * sizeof(u64), s);
    } catch (...) {
        delete ct;
        throw;
    }
    ct->data = as_u64(ct->buf);
    return ct;
}

vr_ciphertext* view_ct(vr_context* ctx, const BufPtr& buf, u64* data, u32 ncomp, u32 level,
                       double scale)
{
    auto* ct = new vr_ciphertext;
    ct->ctx = ctx;
    ct->buf = buf;
    ct->data = data;
    ct->ncomp = ncomp;
    ct->level = level;
    ct->scale = scale;
    return ct;
}

vr_plaintext* new_pt(vr_context* ctx, u32 level, double scale, hipStream_t s)
{
    auto* pt = new vr_plaintext;
    pt->ctx = ctx;
    pt->level = level;
    pt->scale = scale;
    try {
        pt->buf = dev_alloc(ctx, (size_t)(level + 1) * ctx->n * sizeof(u64), s);
    } catch (...) {
        delete pt;
        throw;
    }
    pt->data = as_u64(pt->buf);
    return pt;
}

// ------------------------------------------------------------------ helpers

namespace {

u64 powmod_e(u64 b, u64 e, u64 q)
{
    u64 r = 1 % q;
    b %= q;
    for (; e; e >>= 1) {
        if (e & 1) r = (u64)((u128)r * b % q);
        b = (u64)((u128)b * b % q);
    }
    return r;
}

std::unique_ptr<vr_ciphertext> hold(vr_ciphertext* c) { return std::unique_ptr<vr_ciphertext>(c); }

}  // namespace

u32 galois_element(vr_context* ctx, int32_t step)
{
    i64 r = step % (i64)ctx->slots;
    if (r < 0) r += ctx->slots;
    return (u32)powmod_e(5, (u64)r, 2ull * ctx->n);
}

u64 double_to_mod(double x, u64 q)
{
    if (!std::isfinite(x)) throw Error(VR_EINVAL, "constant is not finite");
    double r = std::round(x);   // half away from zero
    bool neg = r < 0;
    double a = std::fabs(r);
    u64 v;
    if (a < 9223372036854775808.0) {
        v = (u64)a % q;
    } else {
        int e;
        double m = std::frexp(a, &e);              // a = m 2^e, m in [0.5, 1)
        u64 mant = (u64)std::ldexp(m, 53);         // exact 53-bit integer
        v = (u64)((u128)(mant % q) * powmod_e(2, (u64)(e - 53), q) % q);
    }
    return neg && v ? q - v : v;
}

void check_same(const vr_ciphertext* a, const vr_ciphertext* b)
{
    if (a->level != b->level) throw Error(VR_ELEVEL, "operand levels differ");
    if (a->scale != b->scale) throw Error(VR_ESCALE, "operand scales differ");
}

const vr_switch_key& rot_key(const vr_eval_keys* ek, u32 g)
{
    auto it = ek->rot.find(g);
    if (it == ek->rot.end()) throw Error(VR_ENOKEY, "no rotation key for Galois element " + std::to_string(g));
    return it->second;
}

// ------------------------------------------------------------------ server ops

vr_ciphertext* ev_add(vr_context* ctx, const vr_ciphertext* a, const vr_ciphertext* b, bool sub,
                      hipStream_t s)
{
    check_same(a, b);
    if (a->ncomp != b->ncomp) throw Error(VR_EINVAL, "operands have different component counts");
    auto out = hold(new_ct(ctx, a->ncomp, a->level, a->scale, s));
    launch_addsub(ctx, out->data, a->data, b->data, a->ncomp, a->level + 1, sub, s);
    return out.release();
}

vr_ciphertext* ev_mul_const(vr_context* ctx, const vr_ciphertext* a, double c, double c_scale,
                            hipStream_t s)
{
    LimbConsts k;
    for (u32 l = 0; l <= a->level; l++) {
        k.c[l] = double_to_mod(c * c_scale, ctx->mod[l]);
        k.cs[l] = shoup_companion(k.c[l], ctx->mod[l]);
    }
    auto out = hold(new_ct(ctx, a->ncomp, a->level, a->scale * c_scale, s));
    launch_mul_scalar(ctx, out->data, a->data, a->ncomp, a->level + 1, k, s);
    return out.release();
}

vr_ciphertext* ev_add_const(vr_context* ctx, const vr_ciphertext* a, double c, hipStream_t s)
{
    LimbConsts k;
    for (u32 l = 0; l <= a->level; l++) k.c[l] = double_to_mod(c * a->scale, ctx->mod[l]);
    auto out = hold(new_ct(ctx, a->ncomp, a->level, a->scale, s));
    size_t poly = (size_t)(a->level + 1) * ctx->n;
    if (a->ncomp > 1)
        VR_HIP(hipMemcpyAsync(out->data + poly, a->data + poly, (a->ncomp - 1) * poly * sizeof(u64),
                              hipMemcpyDeviceToDevice, s));
    launch_add_scalar(ctx, out->data, a->data, a->level + 1, k, s);
    return out.release();
}

vr_ciphertext* ev_mul_plain(vr_context* ctx, const vr_ciphertext* a, const vr_plaintext* pt,
                            hipStream_t s)
{
    if (pt->level < a->level) throw Error(VR_ELEVEL, "plaintext level below ciphertext level");
    auto out = hold(new_ct(ctx, a->ncomp, a->level, a->scale * pt->scale, s));
    launch_mul_plain(ctx, out->data, a->data, pt->data, a->ncomp, a->level + 1, s);
    return out.release();
}

vr_ciphertext* ev_tensor(vr_context* ctx, const vr_ciphertext* a, const vr_ciphertext* b,
                         hipStream_t s)
{
    if (a->level != b->level) throw Error(VR_ELEVEL, "operand levels differ");
    if (a->ncomp != 2 || b->ncomp != 2) throw Error(VR_EINVAL, "tensor needs 2-component inputs");
    auto out = hold(new_ct(ctx, 3, a->level, a->scale * b->scale, s));
    launch_tensor(ctx, out->data, a->data, b->data, a->level + 1, s);
    return out.release();
}

// key switch of d (nq limbs, evaluation domain) with one key; writes out0/out1
// (nq limbs each) adding add0 (through sigma_g) / add1
static void key_switch(vr_context* ctx, const u64* d, u32 level, const u64* key, u32 g, u64* out0,
                       u64* out1, const u64* add0, const u64* add1, hipStream_t s)
{
    KsShape k = ks_shape(ctx, level);
    const size_t n = ctx->n;
    size_t words = keyswitch_modup_scratch(ctx, level) + (size_t)2 * k.next * n +
                   keyswitch_moddown_scratch(ctx, level, 1);
    BufPtr scratch = dev_alloc(ctx, words * sizeof(u64), s);
    u64* X = as_u64(scratch);
    u64* coef = X + (size_t)k.beta * k.next * n;
    u64* U = coef + (size_t)k.nq * n;
    u64* md = U + (size_t)2 * k.next * n;
    keyswitch_modup(ctx, d, level, X, coef, s);
    keyswitch_inner(ctx, X, d, key, level, g, U, s);
    keyswitch_moddown(ctx, U, level, out0, out1, add0, g, add1, md, s);
}

vr_ciphertext* ev_relin(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* a,
                        hipStream_t s)
{
    if (a->ncomp == 2) {
        auto out = hold(new_ct(ctx, 2, a->level, a->scale, s));
        VR_HIP(hipMemcpyAsync(out->data, a->data, (size_t)2 * (a->level + 1) * ctx->n * sizeof(u64),
                              hipMemcpyDeviceToDevice, s));
        return out.release();
    }
    if (a->ncomp != 3) throw Error(VR_EINVAL, "relinearisation needs 3 components");
    size_t poly = (size_t)(a->level + 1) * ctx->n;
    auto out = hold(new_ct(ctx, 2, a->level, a->scale, s));
    key_switch(ctx, a->data + 2 * poly, a->level, ek->rlk.data, 1, out->data, out->data + poly,
               a->data, a->data + poly, s);
    return out.release();
}

vr_ciphertext* ev_relin_rescale(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* a,
                                hipStream_t s)
{
    if (a->ncomp != 3) throw Error(VR_EINVAL, "relinearisation needs 3 components");
    if (a->level == 0) throw Error(VR_ELEVEL, "no limb left to rescale by");
    const u32 level = a->level;
    KsShape k = ks_shape(ctx, level);
    const size_t n = ctx->n, poly = (size_t)(level + 1) * n;
    auto out = hold(new_ct(ctx, 2, level - 1, a->scale / (double)ctx->mod[level], s));
    size_t words = keyswitch_modup_scratch(ctx, level) + (size_t)2 * k.next * n +
                   keyswitch_moddown_scratch(ctx, level, 1);
    BufPtr scratch = dev_alloc(ctx, words * sizeof(u64), s);
    u64* X = as_u64(scratch);
    u64* coef = X + (size_t)k.beta * k.next * n;
    u64* U = coef + (size_t)k.nq * n;
    u64* md = U + (size_t)2 * k.next * n;
    const u64* d = a->data + 2 * poly;
    keyswitch_modup(ctx, d, level, X, coef, s);
    keyswitch_inner(ctx, X, d, ek->rlk.data, level, 1, U, s);
    keyswitch_moddown_rescale_batch(ctx, U, (u64)2 * k.next * n, 1, level, out->data,
                                    out->data + (size_t)level * n, 0, a->data, a->data + poly, 0, md, s);
    return out.release();
}

void rescale_dense(vr_context* ctx, const u64* in, u64* out, u32 n_polys, u32 level, hipStream_t s)
{
    const size_t n = ctx->n;
    BufPtr tmp = dev_alloc(ctx, ((size_t)n_polys + (size_t)n_polys * level) * n * sizeof(u64), s);
    u64* last = as_u64(tmp);                       // [n_polys][N] coefficient form of limb `level`
    u64* r = last + (size_t)n_polys * n;           // [n_polys][level][N]
    LimbSet ls = poly_limbs(const_cast<u64*>(in), last, n_polys, 1, (u64)(level + 1) * n, (int)level);
    ls.slot0 = level;
    ls.out_dense = 1;
    ntt_inverse(ctx, ls, s);
    // centred last limb reduced to every other modulus, as the NTT loads it
    LimbSet lr = poly_limbs(r, r, n_polys, level, (u64)level * n, (int)level);
    lr.cv_src = last;
    lr.cv_ct_stride = n;
    lr.cv_beta = 1;
    lr.cv_mod0 = level;
    // (c - r) q_l^-1 in the transform's last round where the plan allows
    NttEpilogue& ep = lr.epi;
    ep.a = in;
    ep.a_ct = (u64)2 * (level + 1) * n;
    ep.a_comp = (u64)(level + 1) * n;
    ep.out0 = out;
    ep.out1 = out + (size_t)level * n;
    ep.out_ct = (u64)2 * level * n;
    ep.cmul = ctx->d_rinv_tab + (size_t)level * ctx->nmod();
    if (!ntt_forward(ctx, lr, s)) launch_rescale_finish(ctx, out, in, r, n_polys, level, s);
}

vr_ciphertext* ev_rescale(vr_context* ctx, const vr_ciphertext* a, hipStream_t s)
{
    if (a->level == 0) throw Error(VR_ELEVEL, "no limb left to rescale by");
    auto out = hold(new_ct(ctx, a->ncomp, a->level - 1, a->scale / (double)ctx->mod[a->level], s));
    rescale_dense(ctx, a->data, out->data, a->ncomp, a->level, s);
    return out.release();
}

vr_ciphertext* ev_mod_drop(vr_context* ctx, const vr_ciphertext* a, u32 level, hipStream_t s)
{
    if (level > a->level) throw Error(VR_ELEVEL, "mod_drop cannot raise the level");
    auto out = hold(new_ct(ctx, a->ncomp, level, a->scale, s));
    const u64 src_w = (u64)(a->level + 1) * ctx->n, dst_w = (u64)(level + 1) * ctx->n;
    launch_copy_rows(out->data, dst_w, a->data, src_w, dst_w, a->ncomp, s);
    return out.release();
}

void ev_rotate_many(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* a,
                    const int32_t* steps, size_t k, vr_ciphertext** outs, hipStream_t s)
{
    if (a->ncomp != 2) throw Error(VR_EINVAL, "rotation needs a 2-component ciphertext");
    std::vector<u32> gs(k);
    for (size_t i = 0; i < k; i++) {
        gs[i] = galois_element(ctx, steps[i]);
        if (gs[i] != 1) (void)rot_key(ek, gs[i]);   // fail before any work
    }
    std::vector<std::unique_ptr<vr_ciphertext>> made;
    const u32 level = a->level;
    const size_t n = ctx->n, poly = (size_t)(level + 1) * n;
    KsShape sh = ks_shape(ctx, level);
    BufPtr scratch;
    u64 *X = nullptr, *coef = nullptr, *U = nullptr, *md = nullptr;
    for (size_t i = 0; i < k; i++) {
        made.push_back(hold(new_ct(ctx, 2, level, a->scale, s)));
        vr_ciphertext* o = made.back().get();
        if (gs[i] == 1) {
            VR_HIP(hipMemcpyAsync(o->data, a->data, 2 * poly * sizeof(u64), hipMemcpyDeviceToDevice, s));
            continue;
        }
        if (!X) {   // one ModUp of c1 shared by every rotation (hoisting)
            size_t words = keyswitch_modup_scratch(ctx, level) + (size_t)2 * sh.next * n +
                           keyswitch_moddown_scratch(ctx, level, 1);
            scratch = dev_alloc(ctx, words * sizeof(u64), s);
            X = as_u64(scratch);
            coef = X + (size_t)sh.beta * sh.next * n;
            U = coef + (size_t)sh.nq * n;
            md = U + (size_t)2 * sh.next * n;
            keyswitch_modup(ctx, a->data + poly, level, X, coef, s);
        }
        keyswitch_inner(ctx, X, a->data + poly, rot_key(ek, gs[i]).data, level, gs[i], U, s);
        keyswitch_moddown(ctx, U, level, o->data, o->data + poly, a->data, gs[i], nullptr, md, s);
    }
    for (size_t i = 0; i < k; i++) outs[i] = made[i].release();
}

// ------------------------------------------------------------------ client

vr_plaintext* ev_encode(vr_context* ctx, const double* x_host, size_t n, u32 level, double scale,
                        hipStream_t s)
{
    if (n > ctx->slots) throw Error(VR_EINVAL, "more values than slots");
    if (level > ctx->L) throw Error(VR_ELEVEL, "level above the modulus chain");
    std::unique_ptr<vr_plaintext> pt(new_pt(ctx, level, scale, s));
    BufPtr xd = dev_alloc(ctx, std::max<size_t>(n, 1) * sizeof(double), s);
    if (n) VR_HIP(hipMemcpyAsync(xd->ptr, x_host, n * sizeof(double), hipMemcpyHostToDevice, s));
    encode_to_limbs(ctx, (const double*)xd->ptr, (u32)n, 1, 0, scale, pt->data, level + 1, 0, s);
    ntt_forward(ctx, poly_limbs(pt->data, pt->data, 1, level + 1, (u64)(level + 1) * ctx->n, (int)level), s);
    return pt.release();
}

vr_ciphertext* ev_encrypt(vr_context* ctx, const vr_eval_keys* ek, const vr_plaintext* pt,
                          const Seed256& seed, u64 ct_id, hipStream_t s)
{
    const u32 level = pt->level, nl = level + 1;
    const size_t n = ctx->n;
    BufPtr ints = dev_alloc(ctx, 3 * n * sizeof(i64), s);
    BufPtr limbs = dev_alloc(ctx, (size_t)3 * nl * n * sizeof(u64), s);
    i64* vi = (i64*)ints->ptr;
    launch_sample_ternary(ctx, vi, seed, kPurEncV, ct_id, s);
    launch_sample_gauss(ctx, vi + n, seed, kPurEncE0, ct_id, s);
    launch_sample_gauss(ctx, vi + 2 * n, seed, kPurEncE1, ct_id, s);
    std::vector<u32> mods(nl);
    for (u32 l = 0; l < nl; l++) mods[l] = l;
    u64* L3 = as_u64(limbs);
    for (int k = 0; k < 3; k++) launch_int_to_limbs(ctx, L3 + (size_t)k * nl * n, vi + k * n, mods.data(), nl, s);
    ntt_forward(ctx, poly_limbs(L3, L3, 3, nl, (u64)nl * n, (int)level), s);
    auto out = hold(new_ct(ctx, 2, level, pt->scale, s));
    launch_encrypt_combine(ctx, out->data, L3, L3 + (size_t)nl * n, L3 + (size_t)2 * nl * n, ek->pk,
                           pt->data, nl, s);
    return out.release();
}

}  // namespace vr
