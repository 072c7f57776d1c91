// Context construction: RNS primes, roots of unity, twiddle tables and the
// per-modulus reduction constants, all uploaded to HBM once.
//
// Primes: for each requested bit size b (Q chain first, then the special
// primes), the largest prime q < 2^b with q = 1 mod 2N not taken yet
// (deterministic Miller-Rabin, bases = first twelve primes, exact below 2^64).
// Root: psi = g^((q-1)/2N) for the smallest g >= 2 whose power has psi^N = -1.
// Security: total prime bits <= 218 / 438 / 881 / 1740 for N = 2^13 .. 2^16
// (HE standard 2018 for a ternary secret, 2^16 extrapolated conservatively).
#include <cmath>
#include <cstring>

#include "eval.h"

namespace vr {

namespace {

u64 mulmod_h(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }

u64 powmod_p(u64 b, u64 e, u64 q)
{
    u64 r = 1 % q;
    b %= q;
    for (; e; e >>= 1) {
        if (e & 1) r = mulmod_h(r, b, q);
        b = mulmod_h(b, b, q);
    }
    return r;
}

bool miller_rabin(u64 n)
{
    static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (u64 p : bases) {
        if (n == p) return true;
        if (n % p == 0) return false;
    }
    u64 d = n - 1;
    int s = 0;
    while (!(d & 1)) {
        d >>= 1;
        s++;
    }
    for (u64 a : bases) {
        u64 x = powmod_p(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool witness = true;
        for (int r = 1; r < s && witness; r++) {
            x = mulmod_h(x, x, n);
            if (x == n - 1) witness = false;
        }
        if (witness) return false;
    }
    return true;
}

std::vector<u64> gen_primes(u32 log_n, const std::vector<u32>& bits)
{
    u64 two_n = 2ull << log_n;
    std::vector<u64> out;
    for (u32 b : bits) {
        u64 c = (((1ull << b) - 1) / two_n) * two_n + 1;
        bool found = false;
        for (; c >= (1ull << (b - 1)); c -= two_n) {
            bool taken = false;
            for (u64 t : out) taken |= (t == c);
            if (!taken && miller_rabin(c)) {
                found = true;
                break;
            }
        }
        if (!found) throw Error(VR_EINVAL, "no NTT-friendly prime of the requested size");
        out.push_back(c);
    }
    return out;
}

u64 find_psi(u64 q, u32 log_n)
{
    u64 n = 1ull << log_n;
    for (u64 g = 2;; g++) {
        u64 psi = powmod_p(g, (q - 1) / (2 * n), q);
        if (powmod_p(psi, n, q) == q - 1) return psi;
    }
}

u32 bitrev(u32 x, u32 bits)
{
    u32 r = 0;
    for (u32 i = 0; i < bits; i++, x >>= 1) r = (r << 1) | (x & 1);
    return r;
}

u32 security_bound(u32 log_n)
{
    switch (log_n) {
    case 13: return 218;
    case 14: return 438;
    case 15: return 881;
    case 16: return 1740;
    default: return 0;
    }
}

template <class T>
T* upload(const std::vector<T>& h)
{
    T* d = nullptr;
    VR_HIP(hipMalloc(&d, h.size() * sizeof(T)));
    VR_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
}

}  // namespace

void build_context(vr_context* ctx, const vr_params* p, int device)
{
    if (!p || !p->q_bits || !p->p_bits) throw Error(VR_EINVAL, "null parameters");
    if (p->log_n < 3 || p->log_n > 16) throw Error(VR_EINVAL, "log_n must be in [3, 16]");
    if (p->n_q < 1 || p->n_p < 1 || p->n_q + p->n_p > (u32)kMaxMod)
        throw Error(VR_EINVAL, "bad number of primes (at most 40 in total)");
    if (p->dnum < 1 || p->dnum > p->n_q) throw Error(VR_EINVAL, "dnum must be in [1, n_q]");
    if (std::fabs(p->sigma - 3.2) > 1e-12) throw Error(VR_EINVAL, "sigma must be 3.2");
    std::vector<u32> bits;
    for (u32 i = 0; i < p->n_q; i++) bits.push_back(p->q_bits[i]);
    for (u32 i = 0; i < p->n_p; i++) bits.push_back(p->p_bits[i]);
    for (u32 b : bits)
        if (b < 20 || b > 60) throw Error(VR_EINVAL, "prime sizes must be in [20, 60] bits");

    ctx->device = device;
    ctx->log_n = p->log_n;
    ctx->n = 1u << p->log_n;
    ctx->slots = ctx->n / 2;
    ctx->L = p->n_q - 1;
    ctx->K = p->n_p;
    ctx->dnum = p->dnum;
    ctx->alpha = (p->n_q + p->dnum - 1) / p->dnum;
    if (ctx->alpha > 16 || ctx->K > 16) throw Error(VR_EINVAL, "at most 16 primes per digit");
    if ((p->n_q + ctx->alpha - 1) / ctx->alpha > 16) throw Error(VR_EINVAL, "at most 16 digits");
    ctx->scale = std::ldexp(1.0, 0) * std::pow(2.0, p->log2_scale);
    ctx->mod = gen_primes(p->log_n, bits);
    u32 total = 0;
    for (u64 q : ctx->mod) total += 64 - __builtin_clzll(q);
    u32 bound = security_bound(p->log_n);
    ctx->secure = bound != 0 && total <= bound;
    if (!ctx->secure && !p->allow_insecure)
        throw Error(VR_ESECURITY, "moduli total " + std::to_string(total) +
                                      " bits exceed the 128-bit bound for this N");

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= device)
        throw Error(VR_EDEVICE, "no HIP device available");
    VR_HIP(hipSetDevice(device));
    ctx->arena = std::make_shared<DeviceArena>(device);
    noalloc_register_device(device);   // once per device, this device current

    const u32 n = ctx->n, nmod = ctx->nmod();
    ctx->modq.resize(nmod);
    std::vector<u64> tw((size_t)nmod * n * 2), itw((size_t)nmod * n * 2);
    std::vector<double> twf((size_t)nmod * n), itwf((size_t)nmod * n);
    std::vector<u64> pw(n), ipw(n);
    for (u32 m = 0; m < nmod; m++) {
        u64 q = ctx->mod[m];
        ModQ& mq = ctx->modq[m];
        memset(&mq, 0, sizeof(mq));
        mq.q = q;
        mq.k = 64 - __builtin_clzll(q);
        mq.mu = (u64)(((u128)1 << (2 * mq.k)) / q);
        mq.r64 = (u64)(((u128)1 << 64) % q);
        mq.r64_s = shoup_companion(mq.r64, q);
        mq.one_s = (u64)((((u128)1) << 64) / q);
        mq.ninv = powmod_p(n % q, q - 2, q);
        mq.ninv_s = shoup_companion(mq.ninv, q);
        u64 P = 1;
        for (u32 k = 0; k < ctx->K; k++) P = mulmod_h(P, ctx->mod[ctx->L + 1 + k] % q, q);
        mq.pmod = P;
        mq.pmod_s = shoup_companion(P, q);
        if (m <= ctx->L) {
            mq.pinv = powmod_p(P, q - 2, q);
            mq.pinv_s = shoup_companion(mq.pinv, q);
        }
        u64 psi = find_psi(q, p->log_n);
        u64 ipsi = powmod_p(psi, q - 2, q);
        pw[0] = ipw[0] = 1;
        for (u32 k = 1; k < n; k++) {
            pw[k] = mulmod_h(pw[k - 1], psi, q);
            ipw[k] = mulmod_h(ipw[k - 1], ipsi, q);
        }
        // the inverse's last stage has the single twiddle ipsi^(N/2)
        mq.inw1 = mulmod_h(ipw[n / 2], mq.ninv, q);
        mq.inw1_s = shoup_companion(mq.inw1, q);
        for (u32 k = 0; k < n; k++) {
            u32 e = bitrev(k, p->log_n);
            size_t at = 2 * ((size_t)m * n + k);
            tw[at] = pw[e];
            tw[at + 1] = shoup_companion(pw[e], q);
            itw[at] = ipw[e];
            itw[at + 1] = shoup_companion(ipw[e], q);
            // balanced (-q/2, q/2] copies for the FP64 butterflies (exact below 2^53)
            twf[(size_t)m * n + k] = pw[e] > q / 2 ? -(double)(q - pw[e]) : (double)pw[e];
            itwf[(size_t)m * n + k] = ipw[e] > q / 2 ? -(double)(q - ipw[e]) : (double)ipw[e];
        }
    }
    ctx->d_modq = upload(ctx->modq);
    {
        std::vector<ulonglong2> pinv(nmod), rinv((size_t)(ctx->L + 1) * nmod),
            prinv((size_t)(ctx->L + 1) * nmod), pmod(nmod);
        for (u32 m = 0; m < nmod; m++) {
            const u64 q = ctx->mod[m];
            u64 v = 1 % q;
            for (u32 k = 0; k < ctx->K; k++) v = (u64)((u128)v * (ctx->mod[ctx->L + 1 + k] % q) % q);
            pmod[m] = make_ulonglong2(v, shoup_companion(v, q));
        }
        for (u32 m = 0; m < nmod; m++) pinv[m] = make_ulonglong2(ctx->modq[m].pinv, ctx->modq[m].pinv_s);
        for (u32 l = 0; l <= ctx->L; l++)
            for (u32 i = 0; i < l; i++) {
                const u64 q = ctx->mod[i], c = powmod_p(ctx->mod[l] % q, q - 2, q);
                rinv[(size_t)l * nmod + i] = make_ulonglong2(c, shoup_companion(c, q));
                u64 pq = ctx->mod[l] % q;
                for (u32 k = 0; k < ctx->K; k++) pq = (u64)((u128)pq * (ctx->mod[ctx->L + 1 + k] % q) % q);
                const u64 e = powmod_p(pq, q - 2, q);
                prinv[(size_t)l * nmod + i] = make_ulonglong2(e, shoup_companion(e, q));
            }
        ctx->d_pinv_tab = upload(pinv);
        ctx->d_rinv_tab = upload(rinv);
        ctx->d_prinv_tab = upload(prinv);
        ctx->d_pmod_tab = upload(pmod);
    }
    ctx->d_tw = upload(tw);
    ctx->d_itw = upload(itw);
    ctx->d_twf = upload(twf);
    ctx->d_itwf = upload(itwf);

    // FFT twiddles e^{-2 pi i k / 2N}, k < N, as (re, im) pairs
    std::vector<double> ft(2 * (size_t)n);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (u32 k = 0; k < n; k++) {
        long double ang = -pi * (long double)k / (long double)n;
        ft[2 * k] = (double)cosl(ang);
        ft[2 * k + 1] = (double)sinl(ang);
    }
    ctx->d_fft_tw = upload(ft);
    std::vector<int> gexp(ctx->slots);
    u64 g = 1;
    for (u32 j = 0; j < ctx->slots; j++) {
        gexp[j] = (int)g;
        g = g * 5 % (2ull * n);
    }
    ctx->d_gexp = upload(gexp);
}

void destroy_context_tables(vr_context* ctx)
{
    (void)hipFree(ctx->d_modq);
    (void)hipFree(ctx->d_tw);
    (void)hipFree(ctx->d_itw);
    (void)hipFree(ctx->d_twf);
    (void)hipFree(ctx->d_itwf);
    (void)hipFree(ctx->d_fft_tw);
    (void)hipFree(ctx->d_pinv_tab);
    (void)hipFree(ctx->d_prinv_tab);
    (void)hipFree(ctx->d_pmod_tab);
    (void)hipFree(ctx->d_rinv_tab);
    (void)hipFree(ctx->d_gexp);
    for (auto& kv : ctx->modup_tables)
        (void)hipFree(kv.second.dev), (void)hipFree(kv.second.wt), (void)hipFree(kv.second.wf);
    for (auto& kv : ctx->modup_range_tables)
        (void)hipFree(kv.second.dev), (void)hipFree(kv.second.wt), (void)hipFree(kv.second.wf);
    for (auto& kv : ctx->moddown_tables)
        (void)hipFree(kv.second.dev), (void)hipFree(kv.second.wt), (void)hipFree(kv.second.wf);
    for (auto& kv : ctx->moddown_rs_tables)
        (void)hipFree(kv.second.dev), (void)hipFree(kv.second.wt), (void)hipFree(kv.second.wf);
}

}  // namespace vr
