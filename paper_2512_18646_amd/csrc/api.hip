// C ABI (include/vr.h): argument checks, handle lifetime, error codes.  No C++
// exception crosses this boundary.
#include <cstring>

#include "eval.h"

namespace vr {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

}  // namespace vr

using namespace vr;

#define API_BEGIN try {
#define API_END                                                  \
    }                                                            \
    catch (const vr::Error& e)                                   \
    {                                                            \
        set_last_error(e.what());                                \
        return e.code;                                           \
    }                                                            \
    catch (const std::bad_alloc&)                                \
    {                                                            \
        set_last_error("host allocation failed");                \
        return VR_ENOMEM;                                        \
    }                                                            \
    catch (const std::exception& e)                              \
    {                                                            \
        set_last_error(e.what());                                \
        return VR_EINVAL;                                        \
    }                                                            \
    return VR_OK;

#define REQUIRE(cond, msg) \
    if (!(cond)) throw Error(VR_EINVAL, msg)

namespace vr {

void gen_switch_key(vr_context* ctx, const Seed256& seed, const u64* s_all, const u64* sp_all, u32 g,
                    vr_switch_key& key, hipStream_t st)
{
    const u32 nmod = ctx->nmod();
    const size_t n = ctx->n;
    key.buf = dev_alloc(ctx, (size_t)ctx->dnum * 2 * nmod * n * sizeof(u64), st);
    key.data = as_u64(key.buf);
    BufPtr tmp = dev_alloc(ctx, (n + (size_t)nmod * n) * sizeof(u64), st);
    i64* eint = (i64*)tmp->ptr;
    u64* e = as_u64(tmp) + n;
    std::vector<u32> idx(nmod);
    for (u32 i = 0; i < nmod; i++) idx[i] = i;
    for (u32 j = 0; j < ctx->dnum; j++) {
        u64 obj = (u64)g * 64 + j;
        u64* b = key.data + (size_t)(2 * j) * nmod * n;
        u64* a = key.data + (size_t)(2 * j + 1) * nmod * n;
        launch_sample_uniform(ctx, a, seed, kPurSwkA, obj, idx.data(), idx.data(), nmod, st);
        launch_sample_gauss(ctx, eint, seed, kPurSwkE, obj, st);
        launch_int_to_limbs(ctx, e, eint, idx.data(), nmod, st);
        // every slot is its own modulus index: level = nmod - 1
        LimbSet la = poly_limbs(a, a, 1, nmod, (u64)nmod * n, (int)nmod - 1);
        ntt_forward(ctx, la, st);
        LimbSet le = la;
        le.in = le.out = e;
        ntt_forward(ctx, le, st);
        u32 lo = j * ctx->alpha, hi = std::min((j + 1) * ctx->alpha, ctx->L + 1);
        launch_key_combine(ctx, b, a, e, s_all, sp_all, nmod, lo, hi, st);
    }
}

void add_rotation_keys(vr_context* ctx, const vr_secret_key* sk, vr_eval_keys* ek, const Seed256& seed,
                       const int32_t* steps, size_t n_steps, hipStream_t st)
{
    const u32 nmod = ctx->nmod();
    BufPtr sp;
    for (size_t i = 0; i < n_steps; i++) {
        u32 g = galois_element(ctx, steps[i]);
        if (g == 1 || ek->rot.count(g)) continue;
        if (!sp) sp = dev_alloc(ctx, (size_t)nmod * ctx->n * sizeof(u64), st);
        launch_automorphism(ctx, as_u64(sp), sk->s, 1, nmod, (u64)nmod * ctx->n, g, st);
        vr_switch_key key;
        gen_switch_key(ctx, seed, sk->s, as_u64(sp), g, key, st);
        ek->rot[g] = key;
    }
}

}  // namespace vr

extern "C" {

const char* vr_last_error(void) { return last_error_cstr(); }

vr_status vr_context_create(const vr_params* params, int device, vr_context** out)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(out, "null output");
    std::unique_ptr<vr_context> ctx(new vr_context);
    try {
        build_context(ctx.get(), params, device);
    } catch (...) {
        destroy_context_tables(ctx.get());
        throw;
    }
    *out = ctx.release();
    API_END
}

void vr_context_destroy(vr_context* ctx)
{
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    destroy_context_tables(ctx);
    for (hipEvent_t e : ctx->prof.ev) (void)hipEventDestroy(e);
    delete ctx;
}

vr_status vr_context_moduli(const vr_context* ctx, uint64_t* moduli, size_t cap)
{
    API_BEGIN
    REQUIRE(ctx && moduli, "null argument");
    REQUIRE(cap >= ctx->mod.size(), "capacity too small");
    for (size_t i = 0; i < ctx->mod.size(); i++) moduli[i] = ctx->mod[i];
    API_END
}

vr_status vr_context_info(const vr_context* ctx, uint32_t* info8, double* default_scale)
{
    API_BEGIN
    REQUIRE(ctx && info8, "null argument");
    u32 total = 0;
    for (u64 q : ctx->mod) total += 64 - __builtin_clzll(q);
    u32 v[8] = {ctx->log_n, ctx->slots, ctx->L + 1, ctx->K, ctx->dnum, ctx->alpha,
                ctx->secure ? 1u : 0u, total};
    memcpy(info8, v, sizeof v);
    if (default_scale) *default_scale = ctx->scale;
    API_END
}

vr_status vr_context_set_stream(vr_context* ctx, void* stream)
{
    API_BEGIN
    REQUIRE(ctx, "null context");
    ctx->stream = (hipStream_t)stream;
    API_END
}

vr_status vr_context_set_allocator(vr_context* ctx, void* (*alloc_fn)(size_t, void*, void*),
                                   void (*free_fn)(void*, void*, void*), void* user)
{
    API_BEGIN
    REQUIRE(ctx, "null context");
    REQUIRE((alloc_fn == nullptr) == (free_fn == nullptr), "set both allocator functions or neither");
    ctx->alloc_fn = alloc_fn;
    ctx->free_fn = free_fn;
    ctx->alloc_user = user;
    API_END
}

vr_status vr_context_mem_info(vr_context* ctx, size_t* reserved, size_t* in_use)
{
    API_BEGIN
    REQUIRE(ctx && reserved && in_use, "null argument");
    ctx->arena->usage(reserved, in_use);
    API_END
}

vr_status vr_context_set_tuning(vr_context* ctx, const char* knob, const char* value)
{
    API_BEGIN
    REQUIRE(ctx && knob && value, "null argument");
    std::string k(knob), v(value);
    int mode = -1;
    if (k == "base_convert")
        mode = v == "auto" ? 0 : v == "alu" ? 1 : v == "mfma" ? 2 : v == "fp64" ? 3 : v == "split" ? 4 : -1;
    else if (k == "ntt") {
        mode = v == "auto" ? 0 : v == "fixed" ? 1 : -1;
        if (v.compare(0, 5, "cand:") == 0) mode = 2 + std::stoi(v.substr(5));
    }
    else if (k == "switch_chunk" || k == "ntt_chunk") mode = std::stoi(v);
    else if (k == "conv_prune" || k == "fc_compact" || k == "lincomb_wide" || k == "lincomb_mfma")
        mode = v == "on" ? 0 : v == "off" ? 1 : -1;
    else throw Error(VR_EINVAL, "unknown tuning knob");
    REQUIRE(mode >= 0, "base_convert takes auto, alu, mfma, fp64 or split; ntt takes auto, fixed or cand:k; "
                       "conv_prune, fc_compact, lincomb_wide and lincomb_mfma take on or off");
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->tuning[k] = mode;
    API_END
}

vr_status vr_context_tuning_report(vr_context* ctx, char* buf, size_t cap)
{
    API_BEGIN
    REQUIRE(ctx && buf && cap > 0, "null argument");
    std::string r;
    std::lock_guard<std::mutex> g(ctx->mu);
    auto name = [](int c) {
        return c < 0 ? "untimed" : c == 1 ? "mfma" : c == 2 ? "fp64" : c == 3 ? "split" : "alu";
    };
    for (auto& kv : ctx->modup_tables)
        r += "modup l" + std::to_string(kv.first.first) + " d" + std::to_string(kv.first.second) + " " +
             std::to_string(kv.second.n_in) + "->" + std::to_string(kv.second.n_out) + ": " +
             name(kv.second.choice ? kv.second.choice->load() : -1) + "\n";
    for (auto& kv : ctx->modup_range_tables)
        r += "modup l" + std::to_string(kv.first[0]) + " d" + std::to_string(kv.first[1]) + " [" +
             std::to_string(kv.first[2]) + "," + std::to_string(kv.first[3]) + ")" +
             (kv.first[5] > kv.first[4]
                  ? "+[" + std::to_string(kv.first[4]) + "," + std::to_string(kv.first[5]) + ")"
                  : std::string()) +
             " " + std::to_string(kv.second.n_in) + "->" + std::to_string(kv.second.n_out) + ": " +
             name(kv.second.choice ? kv.second.choice->load() : -1) + "\n";
    for (auto& kv : ctx->moddown_tables)
        r += "moddown l" + std::to_string(kv.first) + " " + std::to_string(kv.second.n_in) + "->" +
             std::to_string(kv.second.n_out) + ": " +
             name(kv.second.choice ? kv.second.choice->load() : -1) + "\n";
    for (auto& kv : ctx->moddown_rs_tables)
        r += "moddown-rescale l" + std::to_string(kv.first / 1024) + " " + std::to_string(kv.second.n_in) + "->" +
             std::to_string(kv.second.n_out) + ": " +
             name(kv.second.choice ? kv.second.choice->load() : -1) + "\n";
    for (int d = 0; d < 2; d++) {
        if (ctx->ntt_plan[d].empty()) continue;
        r += std::string("ntt N=2^") + std::to_string(ctx->log_n) + (d ? " inverse:" : " forward:");
        for (auto& c : ctx->ntt_plan[d])
            r += " {" + std::to_string(c[0]) + "," + std::to_string(c[1]) + "," + std::to_string(c[2]) +
                 (c[3] == 3 ? ",split" : c[3] == 2 ? ",limb" : c[3] ? ",direct" : "") + ",/" + std::to_string(c[4]) + (c[5] == 5 ? ",r32" : "") + "}";
        r += "\n";
    }
    REQUIRE(r.size() < cap, "report buffer too small");
    memcpy(buf, r.c_str(), r.size() + 1);
    API_END
}

vr_status vr_context_trim(vr_context* ctx)
{
    API_BEGIN
    REQUIRE(ctx, "null context");
    ctx->arena->trim();
    API_END
}

// ------------------------------------------------------------------ client

vr_status vr_keygen(vr_context* ctx, const uint64_t* seed_words, const int32_t* rot_steps, size_t n_steps,
                    vr_secret_key** sk_out, vr_eval_keys** ek_out)
{
    if (sk_out) *sk_out = nullptr;
    if (ek_out) *ek_out = nullptr;
    API_BEGIN
    REQUIRE(ctx && sk_out && ek_out && seed_words, "null argument");
    const Seed256 seed = seed_of(seed_words);
    REQUIRE(n_steps == 0 || rot_steps, "null rotation steps");
    hipStream_t st = ctx->stream;
    const u32 nmod = ctx->nmod(), nq = ctx->L + 1;
    const size_t n = ctx->n;
    std::unique_ptr<vr_secret_key> sk(new vr_secret_key);
    std::unique_ptr<vr_eval_keys> ek(new vr_eval_keys);
    sk->ctx = ek->ctx = ctx;
    std::vector<u32> idx(nmod);
    for (u32 i = 0; i < nmod; i++) idx[i] = i;
    BufPtr ints = dev_alloc(ctx, n * sizeof(i64), st);
    i64* xi = (i64*)ints->ptr;
    // secret: ternary, in every modulus
    sk->buf = dev_alloc(ctx, (size_t)nmod * n * sizeof(u64), st);
    sk->s = as_u64(sk->buf);
    launch_sample_ternary(ctx, xi, seed, kPurSk, 0, st);
    launch_int_to_limbs(ctx, sk->s, xi, idx.data(), nmod, st);
    ntt_forward(ctx, poly_limbs(sk->s, sk->s, 1, nmod, (u64)nmod * n, (int)nmod - 1), st);
    // public key (b, a) = (-a s + e, a) over the Q chain
    ek->pk_buf = dev_alloc(ctx, (size_t)2 * nq * n * sizeof(u64), st);
    ek->pk = as_u64(ek->pk_buf);
    u64* pa = ek->pk + (size_t)nq * n;
    launch_sample_uniform(ctx, pa, seed, kPurPkA, 0, idx.data(), idx.data(), nq, st);
    ntt_forward(ctx, poly_limbs(pa, pa, 1, nq, (u64)nq * n, (int)ctx->L), st);
    BufPtr e = dev_alloc(ctx, (size_t)nq * n * sizeof(u64), st);
    launch_sample_gauss(ctx, xi, seed, kPurPkE, 0, st);
    launch_int_to_limbs(ctx, as_u64(e), xi, idx.data(), nq, st);
    ntt_forward(ctx, poly_limbs(as_u64(e), as_u64(e), 1, nq, (u64)nq * n, (int)ctx->L), st);
    launch_key_combine(ctx, ek->pk, pa, as_u64(e), sk->s, nullptr, nq, 0, 0, st);
    // relinearisation key for s^2
    BufPtr s2 = dev_alloc(ctx, (size_t)nmod * n * sizeof(u64), st);
    launch_mul_plain(ctx, as_u64(s2), sk->s, sk->s, 1, nmod, st);
    gen_switch_key(ctx, seed, sk->s, as_u64(s2), 0, ek->rlk, st);
    add_rotation_keys(ctx, sk.get(), ek.get(), seed, rot_steps, n_steps, st);
    VR_HIP(hipStreamSynchronize(st));
    *sk_out = sk.release();
    *ek_out = ek.release();
    API_END
}

vr_status vr_keys_add_rotations(vr_context* ctx, const vr_secret_key* sk, vr_eval_keys* ek,
                                const uint64_t* seed, const int32_t* rot_steps, size_t n_steps)
{
    API_BEGIN
    REQUIRE(ctx && sk && ek && seed, "null argument");
    REQUIRE(n_steps == 0 || rot_steps, "null rotation steps");
    add_rotation_keys(ctx, sk, ek, seed_of(seed), rot_steps, n_steps, ctx->stream);
    VR_HIP(hipStreamSynchronize(ctx->stream));
    API_END
}

vr_status vr_encode(vr_context* ctx, const double* x, size_t n, uint32_t level, double scale,
                    vr_plaintext** out)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && out && (x || n == 0), "null argument");
    REQUIRE(scale > 0, "scale must be positive");
    *out = ev_encode(ctx, x, n, level, scale, ctx->stream);
    API_END
}

vr_status vr_encrypt(vr_context* ctx, const vr_eval_keys* ek, const vr_plaintext* pt,
                     const uint64_t* seed, uint64_t ct_id, vr_ciphertext** out)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && pt && out && seed, "null argument");
    *out = ev_encrypt(ctx, ek, pt, seed_of(seed), ct_id, ctx->stream);
    API_END
}

vr_status vr_decrypt(vr_context* ctx, const vr_secret_key* sk, const vr_ciphertext* ct,
                     vr_plaintext** out)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && sk && ct && out, "null argument");
    std::unique_ptr<vr_plaintext> pt(new_pt(ctx, ct->level, ct->scale, ctx->stream));
    launch_decrypt_combine(ctx, pt->data, ct->data, ct->ncomp, sk->s, ct->level + 1, ctx->stream);
    *out = pt.release();
    API_END
}

vr_status vr_decode(vr_context* ctx, const vr_plaintext* pt, double* out, size_t n)
{
    API_BEGIN
    REQUIRE(ctx && pt && (out || n == 0), "null argument");
    REQUIRE(n <= ctx->slots, "more values than slots");
    hipStream_t st = ctx->stream;
    BufPtr coef = dev_alloc(ctx, (size_t)ctx->n * sizeof(u64), st);
    BufPtr res = dev_alloc(ctx, std::max<size_t>(n, 1) * sizeof(double), st);
    LimbSet ls = poly_limbs(pt->data, as_u64(coef), 1, 1, (u64)(pt->level + 1) * ctx->n, (int)pt->level);
    ls.out_dense = 1;
    ntt_inverse(ctx, ls, st);
    if (n) {
        decode_from_limb0(ctx, as_u64(coef), pt->scale, (double*)res->ptr, (u32)n, st);
        VR_HIP(hipMemcpyAsync(out, res->ptr, n * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    VR_HIP(hipStreamSynchronize(st));
    API_END
}

// ------------------------------------------------------------------ server

vr_status vr_add(vr_context* ctx, const vr_ciphertext* a, const vr_ciphertext* b,
                 vr_ciphertext** out, void* stream)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && a && b && out, "null argument");
    *out = ev_add(ctx, a, b, false, pick_stream(ctx, stream));
    API_END
}

vr_status vr_sub(vr_context* ctx, const vr_ciphertext* a, const vr_ciphertext* b,
                 vr_ciphertext** out, void* stream)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && a && b && out, "null argument");
    *out = ev_add(ctx, a, b, true, pick_stream(ctx, stream));
    API_END
}

vr_status vr_mul_const(vr_context* ctx, const vr_ciphertext* a, double c, double c_scale,
                       vr_ciphertext** out, void* stream)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && a && out, "null argument");
    REQUIRE(c_scale > 0, "constant scale must be positive");
    *out = ev_mul_const(ctx, a, c, c_scale, pick_stream(ctx, stream));
    API_END
}

vr_status vr_add_const(vr_context* ctx, const vr_ciphertext* a, double c, vr_ciphertext** out,
                       void* stream)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && a && out, "null argument");
    *out = ev_add_const(ctx, a, c, pick_stream(ctx, stream));
    API_END
}

vr_status vr_mul_plain(vr_context* ctx, const vr_ciphertext* a, const vr_plaintext* pt,
                       vr_ciphertext** out, void* stream)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && a && pt && out, "null argument");
    *out = ev_mul_plain(ctx, a, pt, pick_stream(ctx, stream));
    API_END
}

vr_status vr_tensor(vr_context* ctx, const vr_ciphertext* a, const vr_ciphertext* b,
                    vr_ciphertext** out, void* stream)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && a && b && out, "null argument");
    *out = ev_tensor(ctx, a, b, pick_stream(ctx, stream));
    API_END
}

vr_status vr_relinearize(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* a,
                         vr_ciphertext** out, void* stream)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && a && out, "null argument");
    *out = ev_relin(ctx, ek, a, pick_stream(ctx, stream));
    API_END
}

vr_status vr_mul(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* a,
                 const vr_ciphertext* b, vr_ciphertext** out, void* stream)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && a && b && out, "null argument");
    hipStream_t s = pick_stream(ctx, stream);
    std::unique_ptr<vr_ciphertext> t(ev_tensor(ctx, a, b, s));
    *out = ev_relin(ctx, ek, t.get(), s);
    API_END
}

vr_status vr_relin_rescale(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* a,
                           vr_ciphertext** out, void* stream)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && a && out, "null argument");
    *out = ev_relin_rescale(ctx, ek, a, pick_stream(ctx, stream));
    API_END
}

vr_status vr_mul_rescale(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* a,
                         const vr_ciphertext* b, vr_ciphertext** out, void* stream)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && a && b && out, "null argument");
    hipStream_t s = pick_stream(ctx, stream);
    std::unique_ptr<vr_ciphertext> t(ev_tensor(ctx, a, b, s));
    *out = ev_relin_rescale(ctx, ek, t.get(), s);
    API_END
}

vr_status vr_rescale(vr_context* ctx, const vr_ciphertext* a, vr_ciphertext** out, void* stream)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && a && out, "null argument");
    *out = ev_rescale(ctx, a, pick_stream(ctx, stream));
    API_END
}

vr_status vr_mod_drop(vr_context* ctx, const vr_ciphertext* a, uint32_t level, vr_ciphertext** out,
                      void* stream)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && a && out, "null argument");
    *out = ev_mod_drop(ctx, a, level, pick_stream(ctx, stream));
    API_END
}

vr_status vr_rotate(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* a, int32_t step,
                    vr_ciphertext** out, void* stream)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && a && out, "null argument");
    ev_rotate_many(ctx, ek, a, &step, 1, out, pick_stream(ctx, stream));
    API_END
}

vr_status vr_rotate_many(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* a,
                         const int32_t* steps, size_t k, vr_ciphertext** outs, void* stream)
{
    if (outs)
        for (size_t i = 0; i < k; i++) outs[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && a && outs && (steps || k == 0), "null argument");
    ev_rotate_many(ctx, ek, a, steps, k, outs, pick_stream(ctx, stream));
    API_END
}

// ------------------------------------------------------------------ parity

vr_status vr_ct_export(vr_context* ctx, const vr_ciphertext* ct, uint64_t* host, size_t cap_words,
                       uint32_t* ncomp, uint32_t* level, double* scale)
{
    API_BEGIN
    REQUIRE(ctx && ct && host, "null argument");
    const size_t words = (size_t)ct->ncomp * (ct->level + 1) * ctx->n;
    REQUIRE(cap_words >= words, "export buffer too small");
    hipStream_t st = ctx->stream;
    BufPtr tmp = dev_alloc(ctx, words * sizeof(u64), st);
    LimbSet ls = poly_limbs(ct->data, as_u64(tmp), ct->ncomp, ct->level + 1,
                            (u64)(ct->level + 1) * ctx->n, (int)ct->level);
    ntt_inverse(ctx, ls, st);
    VR_HIP(hipMemcpyAsync(host, tmp->ptr, words * sizeof(u64), hipMemcpyDeviceToHost, st));
    VR_HIP(hipStreamSynchronize(st));
    if (ncomp) *ncomp = ct->ncomp;
    if (level) *level = ct->level;
    if (scale) *scale = ct->scale;
    API_END
}

vr_status vr_ct_import(vr_context* ctx, const uint64_t* host, uint32_t ncomp, uint32_t level,
                       double scale, vr_ciphertext** out)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && host && out, "null argument");
    REQUIRE(ncomp >= 1 && ncomp <= 3, "ncomp must be 1..3");
    REQUIRE(level <= ctx->L, "level above the modulus chain");
    const size_t words = (size_t)ncomp * (level + 1) * ctx->n;
    for (u32 k = 0; k < ncomp; k++)
        for (u32 l = 0; l <= level; l++) {
            const uint64_t* row = host + ((size_t)k * (level + 1) + l) * ctx->n;
            for (u32 t = 0; t < ctx->n; t++)
                REQUIRE(row[t] < ctx->mod[l], "imported limb value not reduced");
        }
    hipStream_t st = ctx->stream;
    std::unique_ptr<vr_ciphertext> ct(new_ct(ctx, ncomp, level, scale, st));
    VR_HIP(hipMemcpyAsync(ct->data, host, words * sizeof(u64), hipMemcpyHostToDevice, st));
    ntt_forward(ctx, poly_limbs(ct->data, ct->data, ncomp, level + 1, (u64)(level + 1) * ctx->n, (int)level), st);
    VR_HIP(hipStreamSynchronize(st));
    *out = ct.release();
    API_END
}

vr_status vr_pt_export(vr_context* ctx, const vr_plaintext* pt, uint64_t* host, size_t cap_words,
                       uint32_t* level, double* scale)
{
    API_BEGIN
    REQUIRE(ctx && pt && host, "null argument");
    const size_t words = (size_t)(pt->level + 1) * ctx->n;
    REQUIRE(cap_words >= words, "export buffer too small");
    hipStream_t st = ctx->stream;
    BufPtr tmp = dev_alloc(ctx, words * sizeof(u64), st);
    ntt_inverse(ctx, poly_limbs(pt->data, as_u64(tmp), 1, pt->level + 1, words, (int)pt->level), st);
    VR_HIP(hipMemcpyAsync(host, tmp->ptr, words * sizeof(u64), hipMemcpyDeviceToHost, st));
    VR_HIP(hipStreamSynchronize(st));
    if (level) *level = pt->level;
    if (scale) *scale = pt->scale;
    API_END
}

vr_status vr_pt_import(vr_context* ctx, const uint64_t* host, uint32_t level, double scale,
                       vr_plaintext** out)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && host && out, "null argument");
    REQUIRE(level <= ctx->L, "level above the modulus chain");
    const size_t words = (size_t)(level + 1) * ctx->n;
    for (u32 l = 0; l <= level; l++)
        for (u32 t = 0; t < ctx->n; t++)
            REQUIRE(host[(size_t)l * ctx->n + t] < ctx->mod[l], "imported limb value not reduced");
    hipStream_t st = ctx->stream;
    std::unique_ptr<vr_plaintext> pt(new_pt(ctx, level, scale, st));
    VR_HIP(hipMemcpyAsync(pt->data, host, words * sizeof(u64), hipMemcpyHostToDevice, st));
    ntt_forward(ctx, poly_limbs(pt->data, pt->data, 1, level + 1, words, (int)level), st);
    VR_HIP(hipStreamSynchronize(st));
    *out = pt.release();
    API_END
}

vr_status vr_sk_export(vr_context* ctx, const vr_secret_key* sk, int8_t* host, size_t n)
{
    API_BEGIN
    REQUIRE(ctx && sk && host, "null argument");
    REQUIRE(n == ctx->n, "n must equal N");
    hipStream_t st = ctx->stream;
    BufPtr tmp = dev_alloc(ctx, (size_t)ctx->n * sizeof(u64), st);
    LimbSet ls = poly_limbs(sk->s, as_u64(tmp), 1, 1, (u64)ctx->nmod() * ctx->n, (int)ctx->L);
    ls.out_dense = 1;
    ntt_inverse(ctx, ls, st);
    std::vector<u64> h(ctx->n);
    VR_HIP(hipMemcpyAsync(h.data(), tmp->ptr, ctx->n * sizeof(u64), hipMemcpyDeviceToHost, st));
    VR_HIP(hipStreamSynchronize(st));
    u64 q = ctx->mod[0];
    for (u32 t = 0; t < ctx->n; t++) host[t] = h[t] == 0 ? 0 : (h[t] == 1 ? 1 : (h[t] == q - 1 ? -1 : 99));
    API_END
}

vr_status vr_swk_export(vr_context* ctx, const vr_eval_keys* ek, uint32_t galois, uint64_t* host,
                        size_t cap_words)
{
    API_BEGIN
    REQUIRE(ctx && ek && host, "null argument");
    const u32 nmod = ctx->nmod();
    const size_t words = (size_t)ctx->dnum * 2 * nmod * ctx->n;
    REQUIRE(cap_words >= words, "export buffer too small");
    const vr_switch_key& key = galois == 0 ? ek->rlk : rot_key(ek, galois);
    hipStream_t st = ctx->stream;
    BufPtr tmp = dev_alloc(ctx, words * sizeof(u64), st);
    ntt_inverse(ctx, poly_limbs(key.data, as_u64(tmp), ctx->dnum * 2, nmod, (u64)nmod * ctx->n,
                                (int)nmod - 1), st);
    VR_HIP(hipMemcpyAsync(host, tmp->ptr, words * sizeof(u64), hipMemcpyDeviceToHost, st));
    VR_HIP(hipStreamSynchronize(st));
    API_END
}

vr_status vr_ct_meta(const vr_ciphertext* ct, uint32_t* ncomp, uint32_t* level, double* scale)
{
    API_BEGIN
    REQUIRE(ct, "null ciphertext");
    if (ncomp) *ncomp = ct->ncomp;
    if (level) *level = ct->level;
    if (scale) *scale = ct->scale;
    API_END
}

vr_status vr_ntt(vr_context* ctx, uint64_t* data, uint32_t n_limbs, const uint32_t* mod_index,
                 int inverse, void* stream)
{
    API_BEGIN
    REQUIRE(ctx && data && (mod_index || n_limbs == 0), "null argument");
    hipStream_t st = pick_stream(ctx, stream);
    for (u32 i = 0; i < n_limbs; i++) REQUIRE(mod_index[i] < ctx->nmod(), "modulus index out of range");
    // runs of limbs whose modulus index is 0, 1, 2, ... go in one launch
    u32 i = 0;
    while (i < n_limbs) {
        u32 period = 1;
        while (i + period < n_limbs && mod_index[i + period] == mod_index[i] + period) period++;
        u32 reps = 1;
        while (i + (reps + 1) * period <= n_limbs) {
            bool same = true;
            for (u32 k = 0; k < period && same; k++)
                same = mod_index[i + reps * period + k] == mod_index[i + k];
            if (!same) break;
            reps++;
        }
        LimbSet ls = poly_limbs(data + (size_t)i * ctx->n, data + (size_t)i * ctx->n, reps, period,
                                (u64)period * ctx->n, (int)ctx->nmod() - 1);
        ls.slot0 = 0;
        // slot l holds modulus mod_index[i] + l: shift via slot0 and pointer offset
        ls.in = ls.out = data + (size_t)i * ctx->n - (size_t)mod_index[i] * ctx->n;
        ls.slot0 = mod_index[i];
        if (inverse)
            ntt_inverse(ctx, ls, st);
        else
            ntt_forward(ctx, ls, st);
        i += reps * period;
    }
    API_END
}

vr_status vr_profile_start(vr_context* ctx, const char* kernel_class, size_t max_launches)
{
    API_BEGIN
    REQUIRE(ctx && kernel_class, "null argument");
    static const char* names[kProfClasses] = {"ntt", "ks_inner", "base_convert", "lincomb", "moddown",
                                              "tensor"};
    int cls = -1;
    for (int i = 0; i < kProfClasses; i++)
        if (strcmp(kernel_class, names[i]) == 0) cls = i;
    REQUIRE(cls >= 0, "unknown kernel class");
    REQUIRE(max_launches >= 1 && max_launches <= (1u << 20), "max_launches out of range");
    Profiler& p = ctx->prof;
    while (p.ev.size() < 2 * max_launches) {
        hipEvent_t e;
        VR_HIP(hipEventCreate(&e));
        p.ev.push_back(e);
    }
    p.cls = cls;
    p.used = 0;
    p.units = p.launches = 0;
    p.overflow = false;
    API_END
}

vr_status vr_profile_stop(vr_context* ctx, double* total_ms, uint64_t* launches, uint64_t* units,
                          uint32_t* dropped)
{
    API_BEGIN
    REQUIRE(ctx, "null context");
    Profiler& p = ctx->prof;
    p.cls = -1;
    VR_HIP(hipDeviceSynchronize());
    double tot = 0;
    for (size_t i = 0; i + 1 < p.used; i += 2) {
        float ms = 0;
        VR_HIP(hipEventElapsedTime(&ms, p.ev[i], p.ev[i + 1]));
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = p.launches;
    if (units) *units = p.units;
    if (dropped) *dropped = p.overflow ? 1 : 0;
    p.used = 0;
    API_END
}

void vr_free_ciphertext(vr_ciphertext* ct) { delete ct; }
void vr_free_plaintext(vr_plaintext* pt) { delete pt; }
void vr_free_keys(vr_secret_key* sk, vr_eval_keys* ek)
{
    delete sk;
    delete ek;
}

}  // extern "C"
