// A whole encrypted network (conv, optional x^2, optional FC) over n_sets
// image sets as one call, and the same schedule captured once into a HIP
// graph and replayed.  The graph owns its input slab (filled by
// vr_graph_set_inputs), every intermediate buffer and its output slab; a
// replay is one hipGraphLaunch with no host work per kernel.
#include <cstring>

#include "slab.h"

namespace vr {

namespace {

struct CnnDesc {
    u32 C_in, h, w, pad, C_out, k, stride, square;
    std::vector<double> K, bias, fc_bias;
    std::vector<BufPtr> fc_hold;     // keeps the weight plaintexts alive
    const u64* fc_P = nullptr;
    u64 fc_stride = 0;
    double fc_scale = 0;
    u32 fc_out = 0, fc_block = 0;
    u32 w_out() const { return (w + 2 * pad - k) / stride + 1; }
    u32 n_in() const { return C_in * w; }
    u32 n_out() const { return fc_out ? fc_out : C_out * w_out(); }
};

CnnDesc make_desc(vr_context* ctx, const vr_cnn_desc* d, u32 level_in, hipStream_t s)
{
    if (d->C_in < 1 || d->C_out < 1 || d->k < 1 || d->stride < 1 || d->pad >= d->k)
        throw Error(VR_EINVAL, "bad conv shape");
    if (d->w + 2 * d->pad < d->k || d->h + 2 * d->pad < d->k)
        throw Error(VR_EINVAL, "kernel larger than the padded image");
    if (!d->K || !d->bias) throw Error(VR_EINVAL, "null conv weights");
    CnnDesc c;
    c.C_in = d->C_in, c.h = d->h, c.w = d->w, c.pad = d->pad, c.C_out = d->C_out, c.k = d->k;
    c.stride = d->stride, c.square = d->square ? 1 : 0;
    c.K.assign(d->K, d->K + (size_t)d->C_out * d->C_in * d->k * d->k);
    c.bias.assign(d->bias, d->bias + d->C_out);
    const u32 needed = 1 + c.square + (d->fc_w ? 1 : 0);
    if (level_in < needed) throw Error(VR_ELEVEL, "not enough levels for the network");
    if (d->fc_w) {
        if (!d->fc_bias || d->fc_out < 1) throw Error(VR_EINVAL, "FC needs weights, bias and outputs");
        if (d->fc_block < 1 || (d->fc_block & (d->fc_block - 1)) || d->fc_block > ctx->slots)
            throw Error(VR_EINVAL, "FC block must be a power of two <= S");
        const size_t count = (size_t)d->fc_out * c.C_out * c.w_out();
        const u32 nl = level_in - c.square;     // limbs of the FC input (level_in - 1 - square + 1)
        BufPtr hold;
        c.fc_P = fc_weights(ctx, d->fc_w, count, nl, &c.fc_stride, &c.fc_scale, hold, s);
        if (hold) c.fc_hold.push_back(hold);
        for (size_t i = 0; i < count; i++) c.fc_hold.push_back(d->fc_w[i]->buf);
        c.fc_bias.assign(d->fc_bias, d->fc_bias + d->fc_out);
        c.fc_out = d->fc_out;
        c.fc_block = d->fc_block;
    }
    return c;
}

// the network on the slab x of n_sets * C_in * w ciphertexts; outputs set
// after set (n_out() each)
Slab run_cnn(vr_context* ctx, const vr_eval_keys* ek, const CnnDesc& d, const Slab& x, u32 n_sets,
             hipStream_t s)
{
    Slab y = conv_slab(ctx, ek, x, n_sets, d.C_in, d.w, d.pad, d.K.data(), d.bias.data(), d.C_out,
                       d.k, d.stride, s);
    if (d.square) y = layer_square(ctx, ek, y, s);
    if (!d.fc_out) return y;
    const u32 per = d.C_out * d.w_out();
    if (n_sets == 1)
        return fc_slab(ctx, ek, y, d.fc_P, d.fc_stride, d.fc_scale, d.fc_out, d.fc_bias.data(),
                       d.fc_block, s);
    Slab z = new_slab(ctx, n_sets * d.fc_out, 2, y.level - 1, 1.0, s);
    for (u32 st = 0; st < n_sets; st++) {
        Slab ys = y;
        ys.n = per;
        ys.base = y.ct(st * per);
        Slab zs = fc_slab(ctx, ek, ys, d.fc_P, d.fc_stride, d.fc_scale, d.fc_out, d.fc_bias.data(),
                          d.fc_block, s);
        z.scale = zs.scale;
        VR_HIP(hipMemcpyAsync(z.ct(st * d.fc_out), zs.base, (size_t)d.fc_out * zs.stride * sizeof(u64),
                              hipMemcpyDeviceToDevice, s));
    }
    return z;
}

struct CaptureGuard {
    CaptureKeep keep;
    CaptureGuard() { g_capture = &keep; }
    ~CaptureGuard() { g_capture = nullptr; }
};

}  // namespace

}  // namespace vr

struct vr_graph {
    vr_context* ctx = nullptr;
    const vr_eval_keys* ek = nullptr;
    vr::CnnDesc desc;
    vr::u32 n_sets = 0;
    vr::Slab in, out;
    std::vector<vr::BufPtr> keep;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

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

namespace {

void copy_inputs(vr_context* ctx, const Slab& dst, const vr_ciphertext* const* in, size_t n,
                 hipStream_t s)
{
    for (size_t i = 0; i < n; i++) {
        REQUIRE(in[i], "null ciphertext");
        if (in[i]->level != dst.level) throw Error(VR_ELEVEL, "input level differs from the graph's");
        if (in[i]->scale != dst.scale) throw Error(VR_ESCALE, "input scale differs from the graph's");
        if (in[i]->ncomp != 2) throw Error(VR_EINVAL, "inputs must be 2-component");
        VR_HIP(hipMemcpyAsync(dst.ct((u32)i), in[i]->data, dst.stride * sizeof(u64),
                              hipMemcpyDeviceToDevice, s));
    }
    (void)ctx;
}

void release_graph(vr_graph* g)
{
    // replays may still run on callers' streams
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    // later frees of what the graph held (and of output handles) follow the context's stream
    for (auto& b : g->keep) b->stream = g->ctx->stream;
    if (g->out.buf) g->out.buf->stream = g->ctx->stream;
    if (g->in.buf) g->in.buf->stream = g->ctx->stream;
    g->keep.clear();
    g->out = Slab();
    g->in = Slab();
    if (g->cap) (void)hipStreamDestroy(g->cap);
    delete g;
}

}  // namespace

extern "C" {

vr_status vr_cnn_forward(vr_context* ctx, const vr_eval_keys* ek, const vr_cnn_desc* desc,
                         const vr_ciphertext* const* in, uint32_t n_sets, vr_ciphertext** out,
                         void* stream)
{
    API_BEGIN
    REQUIRE(ctx && ek && desc && in && out, "null argument");
    REQUIRE(n_sets >= 1, "no image set");
    hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
    REQUIRE(in[0], "null ciphertext");
    CnnDesc d = make_desc(ctx, desc, in[0]->level, s);
    Slab x = gather(ctx, in, n_sets * d.n_in(), s);
    Slab y = run_cnn(ctx, ek, d, x, n_sets, s);
    to_handles(ctx, y, out);
    API_END
}

vr_status vr_graph_create(vr_context* ctx, const vr_eval_keys* ek, const vr_cnn_desc* desc,
                          const vr_ciphertext* const* in, uint32_t n_sets, vr_graph** out)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && desc && in && out, "null argument");
    REQUIRE(n_sets >= 1, "no image set");
    REQUIRE(!ctx->alloc_fn, "graphs need the built-in allocator");
    REQUIRE(ctx->prof.cls < 0, "stop the kernel profiler before capturing a graph");
    REQUIRE(in[0], "null ciphertext");
    vr_graph* g = new vr_graph;
    g->ctx = ctx;
    g->ek = ek;
    g->n_sets = n_sets;
    try {
        VR_HIP(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
        g->desc = make_desc(ctx, desc, in[0]->level, g->cap);
        const u32 n_in = n_sets * g->desc.n_in();
        g->in = new_slab(ctx, n_in, 2, in[0]->level, in[0]->scale, g->cap);
        copy_inputs(ctx, g->in, in, n_in, g->cap);
        // eager run first: builds and uploads every cached constant table
        (void)run_cnn(ctx, ek, g->desc, g->in, n_sets, g->cap);
        VR_HIP(hipStreamSynchronize(g->cap));
        {
            CaptureGuard guard;
            VR_HIP(hipStreamBeginCapture(g->cap, hipStreamCaptureModeRelaxed));
            try {
                g->out = run_cnn(ctx, ek, g->desc, g->in, n_sets, g->cap);
            } catch (...) {
                hipGraph_t partial = nullptr;
                (void)hipStreamEndCapture(g->cap, &partial);
                if (partial) (void)hipGraphDestroy(partial);
                g->keep = std::move(guard.keep.bufs);
                throw;
            }
            VR_HIP(hipStreamEndCapture(g->cap, &g->graph));
            g->keep = std::move(guard.keep.bufs);
        }
        VR_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    } catch (...) {
        release_graph(g);
        throw;
    }
    *out = g;
    API_END
}

vr_status vr_graph_set_inputs(vr_graph* g, const vr_ciphertext* const* in, size_t n, void* stream)
{
    API_BEGIN
    REQUIRE(g && in, "null argument");
    REQUIRE(n == g->in.n, "input count differs from the graph's");
    copy_inputs(g->ctx, g->in, in, n, stream ? (hipStream_t)stream : g->ctx->stream);
    API_END
}

vr_status vr_graph_launch(vr_graph* g, void* stream)
{
    API_BEGIN
    REQUIRE(g, "null graph");
    VR_HIP(hipGraphLaunch(g->exec, stream ? (hipStream_t)stream : g->ctx->stream));
    API_END
}

vr_status vr_graph_outputs(vr_graph* g, vr_ciphertext** out, size_t cap, size_t* n_out)
{
    if (n_out) *n_out = 0;
    API_BEGIN
    REQUIRE(g && out && n_out, "null argument");
    REQUIRE(cap >= g->out.n, "output capacity too small");
    to_handles(g->ctx, g->out, out);
    *n_out = g->out.n;
    API_END
}

void vr_graph_destroy(vr_graph* g)
{
    if (g) release_graph(g);
}

}  // extern "C"
