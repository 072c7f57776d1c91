// A whole encrypted network (conv, optional x^2, optional FC) over n_sets
// image sets as one call, and the same schedule captured once into a HIP
// graph and replayed.  The graph owns its input slab (filled by
// vr_graph_set_inputs), every intermediate buffer and its output slab; a
// replay is one hipGraphLaunch with no host work per kernel.
#include <cstring>

#include "slab.h"

namespace vr {

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
        c.fc_P = fc_weights(ctx, d->fc_w, count, nl, &c.fc_stride, &c.fc_scale, &c.fc_level, hold, s,
                            &c.fc_rep);
        if (hold) c.fc_hold.push_back(hold);
        for (size_t i = 0; i < count; i++) {
            c.fc_hold.push_back(d->fc_w[i]->buf);
            if (d->fc_w[i]->cbuf) c.fc_hold.push_back(d->fc_w[i]->cbuf);
        }
        c.fc_bias.assign(d->fc_bias, d->fc_bias + d->fc_out);
        c.fc_out = d->fc_out;
        c.fc_block = d->fc_block;
    }
    return c;
}

// the network on the slab x of n_sets * C_in * w ciphertexts; outputs set
// after set (n_out() each): the one-session case of run_cnn_multi
Slab run_cnn(vr_context* ctx, const vr_eval_keys* ek, const CnnDesc& d, const Slab& x, u32 n_sets,
             hipStream_t s)
{
    return run_cnn_multi(ctx, {NetSeg{&d, ek, n_sets}}, x, s);
}

// Sets the thread's capture pool for the guard's lifetime.  The context's
// cache is emptied first so the graph's blocks have the device to themselves.
namespace {

struct CaptureGuard {
    std::shared_ptr<CaptureKeep> keep;
    explicit CaptureGuard(vr_context* ctx)
    {
        ctx->arena->trim();
        keep = std::make_shared<CaptureKeep>();
        keep->arena = ctx->arena;
        keep->release_stream = ctx->stream;
        g_capture = keep;
    }
    ~CaptureGuard() { g_capture.reset(); }
};

bool same_net(const CnnDesc& a, const CnnDesc& b)
{
    return a.C_in == b.C_in && a.h == b.h && a.w == b.w && a.pad == b.pad && a.C_out == b.C_out &&
           a.k == b.k && a.stride == b.stride && a.square == b.square && a.K == b.K && a.bias == b.bias &&
           a.fc_P == b.fc_P && a.fc_stride == b.fc_stride && a.fc_out == b.fc_out &&
           a.fc_block == b.fc_block && a.fc_bias == b.fc_bias;
}

// Networks of a batch with the same description are merged into one
// multi-set evaluation while their inputs together stay under this size.
constexpr size_t kBatchMergeBytes = size_t(2) << 30;

// One request of a batch: a network over its own image sets, or a product
// (column-split, or outer-product when `outer`).
struct BatchReq {
    bool cnn = true;
    bool outer = false;
    CnnDesc desc;
    u32 n_sets = 1;
    u32 m = 0, n = 0, p = 0;
    Slab a, b;        // inputs, owned by the batch (b: the Bbar columns, or B')
    Slab out;
};

// Runs every request: networks with the same description and input level
// and scale as one multi-set evaluation, products of one form at one level
// and scale as one merged schedule.
void run_batch(vr_context* ctx, const vr_eval_keys* ek, std::vector<BatchReq>& reqs, hipStream_t s)
{
    // the previous run's outputs go first, so a run never holds two sets
    for (BatchReq& r : reqs) r.out = Slab();
    std::vector<bool> done(reqs.size(), false);
    for (size_t i = 0; i < reqs.size(); i++) {
        if (done[i] || !reqs[i].cnn) continue;
        std::vector<size_t> grp;
        for (size_t j = i; j < reqs.size(); j++)
            if (!done[j] && reqs[j].cnn && same_net(reqs[i].desc, reqs[j].desc) &&
                reqs[j].a.level == reqs[i].a.level && reqs[j].a.scale == reqs[i].a.scale)
                grp.push_back(j), done[j] = true;
        const u32 per_in = reqs[i].desc.n_in(), per_out = reqs[i].desc.n_out();
        {
            // merge into one multi-set evaluation only while the merged input
            // stays small (the merge copies it); larger requests run alone on
            // their own input slab
            size_t bytes = 0;
            std::vector<size_t> keep;
            for (size_t j : grp) {
                const size_t bj = (size_t)reqs[j].a.n * reqs[j].a.stride * sizeof(u64);
                if (keep.empty() || bytes + bj <= kBatchMergeBytes) keep.push_back(j), bytes += bj;
                else done[j] = false;
            }
            grp.swap(keep);
        }
        u32 sets = 0;
        for (size_t j : grp) sets += reqs[j].n_sets;
        Slab x = reqs[i].a;
        if (grp.size() > 1) {
            x = new_slab(ctx, sets * per_in, 2, reqs[i].a.level, reqs[i].a.scale, s);
            u32 at = 0;
            for (size_t j : grp) {
                VR_HIP(hipMemcpyAsync(x.ct(at), reqs[j].a.base, (size_t)reqs[j].a.n * x.stride * sizeof(u64),
                                      hipMemcpyDeviceToDevice, s));
                at += reqs[j].a.n;
            }
        }
        Slab y = run_cnn(ctx, ek, reqs[i].desc, x, sets, s);
        u32 at = 0;
        for (size_t j : grp) {
            reqs[j].out = y;
            reqs[j].out.n = reqs[j].n_sets * per_out;
            reqs[j].out.base = y.ct(at);
            at += reqs[j].n_sets * per_out;
        }
    }
    for (size_t i = 0; i < reqs.size(); i++) {
        if (done[i]) continue;
        std::vector<size_t> grp;
        std::vector<MatReq> mr;
        for (size_t j = i; j < reqs.size(); j++)
            if (!done[j] && !reqs[j].cnn && reqs[j].outer == reqs[i].outer && reqs[j].a.level == reqs[i].a.level &&
                reqs[j].a.scale * reqs[j].b.scale == reqs[i].a.scale * reqs[i].b.scale) {
                grp.push_back(j), done[j] = true;
                MatReq q;
                q.A = reqs[j].a, q.B = reqs[j].b, q.m = reqs[j].m, q.n = reqs[j].n, q.p = reqs[j].p;
                mr.push_back(q);
            }
        std::vector<Slab> outs = reqs[i].outer ? matmul_outer_multi(ctx, ek, mr, s) : matmul_multi(ctx, ek, mr, s);
        for (size_t g = 0; g < grp.size(); g++) reqs[grp[g]].out = outs[g];
    }
}

}  // namespace

}  // namespace vr

struct vr_graph {
    vr_context* ctx = nullptr;
    const vr_eval_keys* ek = nullptr;
    vr::CnnDesc desc;
    vr::u32 n_sets = 0;
    vr::Slab in, out;
    std::shared_ptr<vr::CaptureKeep> keep;   // the graph's memory
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct vr_batch {
    vr_context* ctx = nullptr;
    const vr_eval_keys* ek = nullptr;
    std::vector<vr::BatchReq> reqs;
    std::shared_ptr<vr::CaptureKeep> keep;   // the graph's memory
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

// A batch request's inputs: the caller's ciphertexts in place when they form
// one slab (as the encryption calls and layer outputs return them; the
// request then shares their allocation, so the caller may release its
// handles), else one gathered copy.  Ciphertexts are never modified.
Slab batch_inputs(vr_context* ctx, const vr_ciphertext* const* in, u32 n, hipStream_t s)
{
    Slab x = gather(ctx, in, n, s);
    if (x.ncomp != 2) throw Error(VR_EINVAL, "inputs must be 2-component");
    return x;
}

void release_graph(vr_graph* g)
{
    // replays may still run on callers' streams
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    // later frees of the input slab and of the description's gathered FC
    // weights (both made on the capture stream) follow the context's stream,
    // and happen before that stream goes; the graph's own blocks return when
    // the last handle into them is gone
    if (g->in.buf) g->in.buf->stream = g->ctx->stream;
    for (BufPtr& b : g->desc.fc_hold)
        if (b && b->stream == g->cap) b->stream = g->ctx->stream;
    g->keep.reset();
    g->out = Slab();
    g->in = Slab();
    g->desc = CnnDesc();
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
            CaptureGuard guard(ctx);
            g->keep = guard.keep;
            VR_HIP(hipStreamBeginCapture(g->cap, hipStreamCaptureModeRelaxed));
            try {
                g->out = run_cnn(ctx, ek, g->desc, g->in, n_sets, g->cap);
            } catch (...) {
                hipGraph_t partial = nullptr;
                (void)hipStreamEndCapture(g->cap, &partial);
                if (partial) (void)hipGraphDestroy(partial);
                throw;
            }
            VR_HIP(hipStreamEndCapture(g->cap, &g->graph));
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

vr_status vr_batch_create(vr_context* ctx, const vr_eval_keys* ek, vr_batch** out)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && out, "null argument");
    vr_batch* b = new vr_batch;
    b->ctx = ctx;
    b->ek = ek;
    *out = b;
    API_END
}

vr_status vr_batch_add_cnn(vr_batch* b, const vr_cnn_desc* desc, const vr_ciphertext* const* in,
                           uint32_t n_sets, uint32_t* req_id)
{
    if (req_id) *req_id = 0;
    API_BEGIN
    REQUIRE(b && desc && in && req_id, "null argument");
    REQUIRE(!b->exec, "batch already captured");
    REQUIRE(n_sets >= 1 && in[0], "no image set");
    hipStream_t s = b->ctx->stream;
    BatchReq r;
    r.cnn = true;
    r.desc = make_desc(b->ctx, desc, in[0]->level, s);
    r.n_sets = n_sets;
    const u32 n = n_sets * r.desc.n_in();
    r.a = batch_inputs(b->ctx, in, n, s);
    b->reqs.push_back(std::move(r));
    *req_id = (uint32_t)b->reqs.size() - 1;
    API_END
}

vr_status vr_batch_add_matmul(vr_batch* b, const vr_ciphertext* const* A, const vr_ciphertext* const* Bbar,
                              uint32_t m, uint32_t n, uint32_t p, uint32_t* req_id)
{
    if (req_id) *req_id = 0;
    API_BEGIN
    REQUIRE(b && A && Bbar && req_id, "null argument");
    REQUIRE(!b->exec, "batch already captured");
    REQUIRE(m >= 1 && n >= 1 && p >= 1 && A[0] && Bbar[0], "empty matrix");
    hipStream_t s = b->ctx->stream;
    BatchReq r;
    r.cnn = false;
    r.m = m, r.n = n, r.p = p;
    r.a = batch_inputs(b->ctx, A, n, s);
    r.b = batch_inputs(b->ctx, Bbar, n, s);
    b->reqs.push_back(std::move(r));
    *req_id = (uint32_t)b->reqs.size() - 1;
    API_END
}

vr_status vr_batch_add_matmul_outer(vr_batch* b, const vr_ciphertext* const* A, const vr_ciphertext* const* B,
                                    uint32_t m, uint32_t n, uint32_t p, uint32_t* req_id)
{
    if (req_id) *req_id = 0;
    API_BEGIN
    REQUIRE(b && A && B && req_id, "null argument");
    REQUIRE(!b->exec, "batch already captured");
    REQUIRE(m >= 1 && n >= 1 && p >= 1 && A[0] && B[0], "empty matrix");
    u32 Pp, R, T;
    outer_tiles(b->ctx, m, p, &Pp, &R, &T);
    hipStream_t s = b->ctx->stream;
    BatchReq r;
    r.cnn = false;
    r.outer = true;
    r.m = m, r.n = n, r.p = p;
    r.a = batch_inputs(b->ctx, A, T * n, s);
    r.b = batch_inputs(b->ctx, B, n, s);
    b->reqs.push_back(std::move(r));
    *req_id = (uint32_t)b->reqs.size() - 1;
    API_END
}

vr_status vr_batch_run(vr_batch* b, void* stream)
{
    API_BEGIN
    REQUIRE(b, "null batch");
    REQUIRE(!b->exec, "batch captured: use vr_batch_launch");
    run_batch(b->ctx, b->ek, b->reqs, stream ? (hipStream_t)stream : b->ctx->stream);
    API_END
}

vr_status vr_batch_capture(vr_batch* b)
{
    API_BEGIN
    REQUIRE(b, "null batch");
    REQUIRE(!b->exec, "batch already captured");
    REQUIRE(!b->reqs.empty(), "empty batch");
    REQUIRE(!b->ctx->alloc_fn, "graphs need the built-in allocator");
    REQUIRE(b->ctx->prof.cls < 0, "stop the kernel profiler before capturing a graph");
    VR_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    VR_HIP(hipStreamSynchronize(b->ctx->stream));
    run_batch(b->ctx, b->ek, b->reqs, b->cap);   // eager: builds and tunes every cached constant
    VR_HIP(hipStreamSynchronize(b->cap));
    // release the eager outputs now: nothing allocated before the capture may
    // be freed while it records
    for (auto& r : b->reqs) r.out = Slab();
    {
        CaptureGuard guard(b->ctx);
        b->keep = guard.keep;
        VR_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
        try {
            run_batch(b->ctx, b->ek, b->reqs, b->cap);
        } catch (...) {
            hipGraph_t partial = nullptr;
            (void)hipStreamEndCapture(b->cap, &partial);
            if (partial) (void)hipGraphDestroy(partial);
            throw;
        }
        VR_HIP(hipStreamEndCapture(b->cap, &b->graph));
    }
    VR_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    API_END
}

vr_status vr_batch_launch(vr_batch* b, void* stream)
{
    API_BEGIN
    REQUIRE(b && b->exec, "batch not captured");
    VR_HIP(hipGraphLaunch(b->exec, stream ? (hipStream_t)stream : b->ctx->stream));
    API_END
}

vr_status vr_batch_outputs(vr_batch* b, uint32_t req_id, vr_ciphertext** out, size_t cap, size_t* n_out)
{
    if (n_out) *n_out = 0;
    API_BEGIN
    REQUIRE(b && out && n_out, "null argument");
    REQUIRE(req_id < b->reqs.size(), "unknown request");
    const Slab& o = b->reqs[req_id].out;
    REQUIRE(o.base, "batch not run yet");
    REQUIRE(cap >= o.n, "output capacity too small");
    to_handles(b->ctx, o, out);
    *n_out = o.n;
    API_END
}

void vr_batch_destroy(vr_batch* b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto& r : b->reqs) {
        if (r.out.buf && !r.out.buf->cap) r.out.buf->stream = b->ctx->stream;
        if (r.a.buf) r.a.buf->stream = b->ctx->stream;
        if (r.b.buf) r.b.buf->stream = b->ctx->stream;
    }
    b->reqs.clear();
    b->keep.reset();
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

}  // extern "C"
