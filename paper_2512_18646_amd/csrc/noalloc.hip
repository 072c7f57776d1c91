// Rotation of a ciphertext held in caller-owned device memory, with every
// key-switching intermediate (ModUp digits, the inner product's sums, ModDown's
// scratch) in one fixed device array of the library instead of allocated
// buffers.  It is for callers that cannot allocate device memory: code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
//
// The array is a file-scope __device__ array; each GPU the library runs on
// holds its own copy at its own address until the process ends.  Host code
// never passes the array's name to a kernel or copy (on the host the name is
// a stand-in, not a device address): its device address is taken once per
// device with hipGetSymbolAddress when a context is created on that device
// (that device current), kept per device, and only that address is used.
//
// Calls on one GPU share its array, so two calls that overlap on one GPU (on
// different streams, or from different threads) race; calls on one stream
// run one after another and are safe.  Nothing in the array needs to start at
// zero: every word a call reads there was written earlier by the same call.
#include <map>
#include <mutex>

#include "eval.h"

namespace vr {

namespace {

__device__ __align__(256) u64 scratch[kNoAllocScratchBytes / sizeof(u64)];

std::mutex g_mu;
std::map<int, u64*> g_ptr;   // device -> device address of its copy of `scratch`

}  // namespace

void noalloc_register_device(int device)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (g_ptr.count(device)) return;
    void* p = nullptr;
    hipError_t rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (rc != hipSuccess || !p)
        throw Error(VR_EDEVICE, std::string("no-allocation scratch: hipGetSymbolAddress failed: ") +
                                    hipGetErrorString(rc));
    g_ptr[device] = (u64*)p;
}

namespace {

u64* scratch_of(int device)
{
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_ptr.find(device);
    if (it == g_ptr.end()) throw Error(VR_EDEVICE, "no-allocation scratch: device not registered");
    return it->second;
}

// Everything a rotation at `level` would build on first use (NTT plans,
// base-conversion tables and the choice of their kernel) must exist already:
// building it allocates.
void require_prepared(vr_context* ctx, u32 level)
{
    std::lock_guard<std::mutex> g(ctx->mu);
    auto mode = [&](const char* k) {
        auto it = ctx->tuning.find(k);
        return it == ctx->tuning.end() ? 0 : it->second;
    };
    const char* hint = "; run one allocating operation at this level first (e.g. vr_rotate)";
    if (mode("ntt") == 0 && (ctx->ntt_plan[0].empty() || ctx->ntt_plan[1].empty()))
        throw Error(VR_EINVAL, std::string("no-allocation rotation: the NTT plans are not tuned yet") + hint);
    const bool conv_auto = mode("base_convert") == 0;
    if (ctx->alpha > 1) {
        const u32 beta = (level + ctx->alpha) / ctx->alpha;
        for (u32 j = 0; j < beta; j++) {
            auto it = ctx->modup_tables.find(std::make_pair((int)level, (int)j));
            if (it == ctx->modup_tables.end() || (conv_auto && it->second.choice->load() < 0))
                throw Error(VR_EINVAL, std::string("no-allocation rotation: ModUp tables of this level are "
                                                   "not built yet") + hint);
        }
    }
    if (ctx->K > 1) {
        auto it = ctx->moddown_tables.find((int)level);
        if (it == ctx->moddown_tables.end() || (conv_auto && it->second.choice->load() < 0))
            throw Error(VR_EINVAL, std::string("no-allocation rotation: the ModDown table of this level is "
                                               "not built yet") + hint);
    }
}

}  // namespace

size_t noalloc_rotate_words(vr_context* ctx, u32 level)
{
    KsShape sh = ks_shape(ctx, level);
    return keyswitch_modup_scratch(ctx, level) + (size_t)2 * sh.next * ctx->n +
           keyswitch_moddown_scratch(ctx, level, 1);
}

}  // namespace vr

using namespace vr;

extern "C" vr_status vr_rotate_noalloc(vr_context* ctx, const vr_eval_keys* ek, const uint64_t* in,
                                       uint32_t level, int32_t step, uint64_t* out, void* stream)
{
    try {
        if (!ctx || !ek || !in || !out) throw Error(VR_EINVAL, "null argument");
        if (level > ctx->L) throw Error(VR_ELEVEL, "level above the modulus chain");
        const size_t n = ctx->n, poly = (size_t)(level + 1) * n;
        if (in < out + 2 * poly && out < in + 2 * poly) throw Error(VR_EINVAL, "input and output overlap");
        const size_t words = noalloc_rotate_words(ctx, level);
        if (words * sizeof(u64) > kNoAllocScratchBytes)
            throw Error(VR_EINVAL, "no-allocation rotation: key switching at this level needs " +
                                       std::to_string(words * sizeof(u64)) + " bytes of scratch, above the " +
                                       std::to_string(kNoAllocScratchBytes) + "-byte array");
        hipStream_t s = pick_stream(ctx, stream);
        const u32 g = galois_element(ctx, step);
        if (g == 1) {
            VR_HIP(hipMemcpyAsync(out, in, 2 * poly * sizeof(u64), hipMemcpyDeviceToDevice, s));
            return VR_OK;
        }
        const vr_switch_key& key = rot_key(ek, g);
        require_prepared(ctx, level);
        KsShape sh = ks_shape(ctx, level);
        u64* X = scratch_of(ctx->device);
        u64* coef = X + (size_t)sh.beta * sh.next * n;
        u64* U = coef + (size_t)sh.nq * n;
        u64* md = U + (size_t)2 * sh.next * n;
        keyswitch_modup(ctx, in + poly, level, X, coef, s);
        keyswitch_inner(ctx, X, in + poly, key.data, level, g, U, s);
        keyswitch_moddown(ctx, U, level, out, out + poly, in, g, nullptr, md, s);
        return VR_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return VR_EINVAL;
    }
}
