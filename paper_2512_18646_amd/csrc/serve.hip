// Continuous-batching serving loop for encrypted inference requests.
//
// A request is one image set (the C_in*w column ciphertexts of up to B'
// images, the paper's mini-batch of "Secure Inference") for a registered model
// (conv layer, optionally followed by the x^2 activation and an FC layer)
// under a session whose evaluation keys stay resident in HBM.  A worker thread
// forms "waves": the oldest pending request plus every later pending request
// that can be evaluated stage by stage beside it (same level and scale, models
// with the same conv kernel size, x^2 and FC level; sessions and networks may
// differ), while the wave is under max_batch requests and the device-memory
// estimate of the in-flight waves stays under the budget.  A wave runs as one
// evaluation (run_cnn_multi): the stages that do not depend on the keys
// (ModUp, ModDown, NTTs, rescale, tensor) run once over every request's
// ciphertexts, the key-switch inner products once per session, the linear
// combinations and weight products once per network.  Requests that arrive
// while earlier waves are on the GPU join the next wave; waves alternate
// between two streams so consecutive waves overlap on the device.  Each
// request's output limbs are the same alone or in a wave: every ciphertext's
// arithmetic is independent of the wave's composition.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>

#include "slab.h"

namespace vr {

namespace {

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// A registered network: its description with owned copies of the weights
// (the FC weight plaintexts are the caller's and must outlive the server).
struct Model {
    u32 C_in, h, w, pad, C_out, k, stride;
    bool square;
    std::vector<double> K, bias, fc_bias;
    std::vector<const vr_plaintext*> fc_w;
    u32 fc_out = 0, fc_block = 0;
    u32 n_cols() const { return C_in * w; }
    u32 w_out() const { return (w + 2 * pad - k) / stride + 1; }
    u32 n_out() const { return fc_out ? fc_out : C_out * w_out(); }
    u32 levels() const { return 1 + (square ? 1 : 0) + (fc_out ? 1 : 0); }
    vr_cnn_desc desc() const
    {
        vr_cnn_desc d;
        d.C_in = C_in, d.h = h, d.w = w, d.pad = pad, d.C_out = C_out, d.k = k, d.stride = stride;
        d.K = K.data(), d.bias = bias.data(), d.square = square ? 1 : 0;
        d.fc_w = fc_out ? fc_w.data() : nullptr;
        d.fc_bias = fc_out ? fc_bias.data() : nullptr;
        d.fc_out = fc_out, d.fc_block = fc_block;
        return d;
    }
};

struct Request {
    u64 ticket = 0, session = 0;
    u32 model = 0, level = 0, images = 0;
    double scale = 0;
    std::vector<BufPtr> bufs;      // keep the inputs alive
    std::vector<u64*> data;
    hipEvent_t ready = nullptr;    // inputs written (recorded on the client's stream)
    size_t bytes = 0;
    double t_submit = 0, t_done = 0;
    int state = 0;                 // 0 pending, 1 running, 2 done, 3 failed
    vr_status err = VR_OK;
    std::string msg;
    Slab out;                      // view of the wave's output slab
};

struct Wave {
    hipEvent_t done = nullptr;
    std::vector<Request*> reqs;
    Slab y;
    std::vector<u32> off, cnt;    // request i's outputs: y ciphertexts [off[i], off[i] + cnt[i])
};

}  // namespace

}  // namespace vr

struct vr_server {
    vr_context* ctx = nullptr;
    size_t budget = 0, used = 0, resident = 0;
    vr::u32 max_batch = 1;
    std::map<vr::u64, const vr_eval_keys*> sessions;
    vr::u64 next_session = 1, next_ticket = 1;
    std::deque<vr::Model> models;   // stable references while waves run
    std::map<vr::u64, std::unique_ptr<vr::Request>> reqs;
    std::deque<vr::Request*> pending;
    std::deque<vr::Wave> inflight;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::thread worker;
    bool stop = false;
    hipStream_t streams[2] = {nullptr, nullptr};
    vr::u64 waves = 0, batched_requests = 0;
    std::vector<double> lat_ms;
    vr::u64 images_done = 0;
    double t_first = -1, t_last = 0;
};

namespace vr {

namespace {

size_t key_bytes(vr_context* ctx, const vr_eval_keys* ek)
{
    size_t one = (size_t)ctx->dnum * 2 * ctx->nmod() * ctx->n * sizeof(u64);
    return one * (1 + ek->rot.size()) + (size_t)2 * (ctx->L + 1) * ctx->n * sizeof(u64);
}

// Upper estimate of the device bytes one request holds while its wave runs.
size_t request_bytes(vr_context* ctx, const Model& m, u32 level)
{
    const size_t N = ctx->n;
    auto ks = [&](u32 lv) {
        KsShape k = ks_shape(ctx, lv);
        return ((size_t)k.beta * k.next + k.nq + 2 * k.next + 2 * (ctx->K + k.nq)) * N * 8;
    };
    const size_t ct = (size_t)2 * (level + 1) * N * 8;
    const size_t conv_out = (size_t)m.C_out * m.w_out();
    size_t b = (size_t)m.n_cols() * (ct * (m.k + 1) + ks(level));
    b += conv_out * ct * 2;
    if (m.square) b += conv_out * (ct * 4 + ks(level - 1));
    if (m.fc_out) b += (size_t)m.fc_out * (ct * 2 + ks(level - 2));
    return b;
}

// Requests that can share one wave: same level and scale, and models whose
// evaluations line up stage by stage (conv kernel size, x^2, FC presence and
// the level the FC runs at); sessions and networks may differ.
bool wave_compatible(const vr_server* srv, const Request* a, const Request* b)
{
    if (a->level != b->level || a->scale != b->scale) return false;
    const Model& ma = srv->models[a->model];
    const Model& mb = srv->models[b->model];
    auto fc_level = [&](const Model& m, u32 level) {
        return std::min(level - (m.square ? 1u : 0u) - 1u, m.fc_w[0]->level);
    };
    return ma.k == mb.k && ma.square == mb.square && (ma.fc_out != 0) == (mb.fc_out != 0) &&
           (!ma.fc_out || (fc_level(ma, a->level) == fc_level(mb, b->level) &&
                           ma.fc_w[0]->scale == mb.fc_w[0]->scale));
}

// One wave: requests ordered by FC block (decreasing), model and session so
// that each (model, session) pair is one segment of consecutive image sets;
// their columns copied into one slab and evaluated by run_cnn_multi.
void run_wave(vr_server* srv, Wave& wv, hipStream_t s)
{
    vr_context* ctx = srv->ctx;
    std::stable_sort(wv.reqs.begin(), wv.reqs.end(), [&](const Request* a, const Request* b) {
        const Model& ma = srv->models[a->model];
        const Model& mb = srv->models[b->model];
        if (ma.fc_block != mb.fc_block) return ma.fc_block > mb.fc_block;
        if (a->model != b->model) return a->model < b->model;
        return a->session < b->session;
    });
    Request* r0 = wv.reqs[0];
    std::map<u32, CnnDesc> descs;
    std::vector<NetSeg> segs;
    u32 n_in = 0;
    for (Request* r : wv.reqs) {
        VR_HIP(hipStreamWaitEvent(s, r->ready, 0));
        auto it = descs.find(r->model);
        if (it == descs.end()) {
            const vr_cnn_desc dd = srv->models[r->model].desc();
            it = descs.emplace(r->model, make_desc(ctx, &dd, r0->level, s)).first;
        }
        const vr_eval_keys* ek = srv->sessions.at(r->session);
        if (!segs.empty() && segs.back().d == &it->second && segs.back().ek == ek)
            segs.back().n_sets++;
        else
            segs.push_back(NetSeg{&it->second, ek, 1});
        n_in += it->second.n_in();
    }
    Slab x = new_slab(ctx, n_in, 2, r0->level, r0->scale, s);
    u32 at = 0, out_at = 0;
    for (Request* r : wv.reqs) {
        const CnnDesc& d = descs.at(r->model);
        for (u32 c = 0; c < d.n_in(); c++)
            VR_HIP(hipMemcpyAsync(x.ct(at + c), r->data[c], x.stride * sizeof(u64), hipMemcpyDeviceToDevice, s));
        at += d.n_in();
        wv.off.push_back(out_at);
        wv.cnt.push_back(d.n_out());
        out_at += d.n_out();
    }
    wv.y = run_cnn_multi(ctx, segs, x, s);
    VR_HIP(hipEventCreateWithFlags(&wv.done, hipEventDisableTiming));
    VR_HIP(hipEventRecord(wv.done, s));
}

void retire(vr_server* srv)
{
    // caller holds srv->mu
    while (!srv->inflight.empty()) {
        Wave& wv = srv->inflight.front();
        hipError_t q = hipEventQuery(wv.done);
        if (q == hipErrorNotReady) break;
        double t = now_ms();
        // the wave is complete: later frees of its outputs follow the client's stream
        if (wv.y.buf) wv.y.buf->stream = srv->ctx->stream;
        for (size_t i = 0; i < wv.reqs.size(); i++) {
            Request* r = wv.reqs[i];
            if (q == hipSuccess) {
                r->state = 2;
                r->out = wv.y;
                r->out.n = wv.cnt[i];
                r->out.base = wv.y.ct(wv.off[i]);
            } else {
                r->state = 3;
                r->err = VR_EDEVICE;
                r->msg = hipGetErrorString(q);
            }
            r->t_done = t;
            srv->used -= r->bytes;
            r->bufs.clear();
            r->data.clear();
            (void)hipEventDestroy(r->ready);
            r->ready = nullptr;
            srv->lat_ms.push_back(t - r->t_submit);
            srv->images_done += r->images;
            if (srv->t_first < 0 || r->t_submit < srv->t_first) srv->t_first = r->t_submit;
            srv->t_last = t;
        }
        (void)hipEventDestroy(wv.done);
        srv->inflight.pop_front();
        srv->done_cv.notify_all();
    }
}

void worker_loop(vr_server* srv)
{
    (void)hipSetDevice(srv->ctx->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    while (true) {
        retire(srv);
        if (srv->stop && srv->pending.empty() && srv->inflight.empty()) break;
        bool launched = false;
        if (!srv->pending.empty() && srv->inflight.size() < 2) {
            Request* head = srv->pending.front();
            const size_t cap = srv->budget > srv->resident ? srv->budget - srv->resident : 0;
            if (head->bytes > cap) {
                // sessions registered after the submit left no room for it
                srv->pending.pop_front();
                head->state = 3;
                head->err = VR_EBUSY;
                head->msg = "request no longer fits the memory budget";
                head->bufs.clear();
                head->data.clear();
                (void)hipEventDestroy(head->ready);
                head->ready = nullptr;
                srv->done_cv.notify_all();
                continue;
            }
            if (srv->used + head->bytes <= cap) {
                Wave wv;
                wv.reqs.push_back(head);
                srv->used += head->bytes;
                srv->pending.pop_front();
                for (auto it = srv->pending.begin(); it != srv->pending.end();) {
                    Request* r = *it;
                    if (wv.reqs.size() >= srv->max_batch) break;
                    if (wave_compatible(srv, r, head) && srv->used + r->bytes <= cap) {
                        wv.reqs.push_back(r);
                        srv->used += r->bytes;
                        it = srv->pending.erase(it);
                    } else {
                        ++it;
                    }
                }
                for (Request* r : wv.reqs) r->state = 1;
                hipStream_t s = srv->streams[srv->waves % 2];
                srv->waves++;
                srv->batched_requests += wv.reqs.size();
                lk.unlock();
                std::string err;
                vr_status code = VR_OK;
                try {
                    run_wave(srv, wv, s);
                } catch (const Error& e) {
                    code = e.code;
                    err = e.what();
                } catch (const std::exception& e) {
                    code = VR_EINVAL;
                    err = e.what();
                }
                lk.lock();
                if (code != VR_OK) {
                    double t = now_ms();
                    // drain what the failed wave queued before releasing its inputs
                    (void)hipStreamSynchronize(s);
                    for (Request* r : wv.reqs) {
                        r->state = 3;
                        r->err = code;
                        r->msg = err;
                        r->t_done = t;
                        srv->used -= r->bytes;
                        r->bufs.clear();
                        (void)hipEventDestroy(r->ready);
                        r->ready = nullptr;
                    }
                    srv->done_cv.notify_all();
                } else {
                    srv->inflight.push_back(wv);
                }
                launched = true;
            }
        }
        if (launched) continue;
        if (!srv->inflight.empty()) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(50));
            lk.lock();
        } else {
            srv->cv.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

}  // namespace

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

extern "C" {

vr_status vr_srv_create(vr_context* ctx, size_t hbm_budget_bytes, uint32_t max_batch, vr_server** out)
{
    if (out) *out = nullptr;
    API_BEGIN
    REQUIRE(ctx && out, "null argument");
    REQUIRE(max_batch >= 1, "max_batch must be >= 1");
    std::unique_ptr<vr_server> srv(new vr_server);
    srv->ctx = ctx;
    srv->budget = hbm_budget_bytes;
    srv->max_batch = max_batch;
    VR_HIP(hipStreamCreateWithFlags(&srv->streams[0], hipStreamNonBlocking));
    VR_HIP(hipStreamCreateWithFlags(&srv->streams[1], hipStreamNonBlocking));
    vr_server* raw = srv.get();
    srv->worker = std::thread([raw] { worker_loop(raw); });
    *out = srv.release();
    API_END
}

void vr_srv_destroy(vr_server* srv)
{
    if (!srv) return;
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    for (auto& kv : srv->reqs) kv.second->out = Slab();
    (void)hipStreamSynchronize(srv->streams[0]);
    (void)hipStreamSynchronize(srv->streams[1]);
    srv->reqs.clear();
    (void)hipStreamDestroy(srv->streams[0]);
    (void)hipStreamDestroy(srv->streams[1]);
    delete srv;
}

vr_status vr_srv_register_session(vr_server* srv, const vr_eval_keys* ek, uint64_t* session_id)
{
    if (session_id) *session_id = 0;
    API_BEGIN
    REQUIRE(srv && ek && session_id, "null argument");
    std::lock_guard<std::mutex> g(srv->mu);
    size_t kb = key_bytes(srv->ctx, ek);
    if (srv->resident + kb > srv->budget) throw Error(VR_EBUSY, "session keys exceed the memory budget");
    srv->resident += kb;
    u64 id = srv->next_session++;
    srv->sessions[id] = ek;
    *session_id = id;
    API_END
}

vr_status vr_srv_register_conv_model(vr_server* srv, uint32_t C_in, uint32_t h, uint32_t w,
                                     uint32_t pad, const double* K, const double* bias,
                                     uint32_t C_out, uint32_t k, uint32_t stride, uint32_t square,
                                     uint32_t* model_id)
{
    if (model_id) *model_id = 0;
    API_BEGIN
    REQUIRE(srv && K && bias && model_id, "null argument");
    REQUIRE(C_in >= 1 && C_out >= 1 && k >= 1 && stride >= 1 && pad < k, "bad conv shape");
    REQUIRE(w + 2 * pad >= k && h + 2 * pad >= k, "kernel larger than the padded image");
    Model m;
    m.C_in = C_in, m.h = h, m.w = w, m.pad = pad, m.C_out = C_out, m.k = k, m.stride = stride;
    m.square = square != 0;
    m.K.assign(K, K + (size_t)C_out * C_in * k * k);
    m.bias.assign(bias, bias + C_out);
    std::lock_guard<std::mutex> g(srv->mu);
    srv->models.push_back(m);
    *model_id = (u32)srv->models.size() - 1;
    API_END
}

vr_status vr_srv_register_model(vr_server* srv, const vr_cnn_desc* d, uint32_t* model_id)
{
    if (model_id) *model_id = 0;
    API_BEGIN
    REQUIRE(srv && d && model_id && d->K && d->bias, "null argument");
    REQUIRE(d->C_in >= 1 && d->C_out >= 1 && d->k >= 1 && d->stride >= 1 && d->pad < d->k, "bad conv shape");
    REQUIRE(d->w + 2 * d->pad >= d->k && d->h + 2 * d->pad >= d->k, "kernel larger than the padded image");
    Model m;
    m.C_in = d->C_in, m.h = d->h, m.w = d->w, m.pad = d->pad, m.C_out = d->C_out, m.k = d->k;
    m.stride = d->stride, m.square = d->square != 0;
    m.K.assign(d->K, d->K + (size_t)d->C_out * d->C_in * d->k * d->k);
    m.bias.assign(d->bias, d->bias + d->C_out);
    if (d->fc_w) {
        REQUIRE(d->fc_bias && d->fc_out >= 1, "FC needs weights, bias and outputs");
        REQUIRE(d->fc_block >= 1 && (d->fc_block & (d->fc_block - 1)) == 0 && d->fc_block <= srv->ctx->slots,
                "FC block must be a power of two <= S");
        const size_t count = (size_t)d->fc_out * d->C_out * m.w_out();
        for (size_t i = 0; i < count; i++) REQUIRE(d->fc_w[i], "null weight plaintext");
        m.fc_w.assign(d->fc_w, d->fc_w + count);
        m.fc_bias.assign(d->fc_bias, d->fc_bias + d->fc_out);
        m.fc_out = d->fc_out;
        m.fc_block = d->fc_block;
    }
    std::lock_guard<std::mutex> g(srv->mu);
    srv->models.push_back(m);
    *model_id = (u32)srv->models.size() - 1;
    API_END
}

vr_status vr_srv_submit(vr_server* srv, uint64_t session_id, uint32_t model_id,
                        const vr_ciphertext* const* in, size_t n_in, uint32_t n_images,
                        uint64_t* ticket)
{
    if (ticket) *ticket = 0;
    API_BEGIN
    REQUIRE(srv && in && ticket, "null argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    REQUIRE(srv->sessions.count(session_id), "unknown session");
    REQUIRE(model_id < srv->models.size(), "unknown model");
    const Model& m = srv->models[model_id];
    REQUIRE(n_in == m.n_cols(), "input count must equal C_in * w of the model");
    std::unique_ptr<Request> r(new Request);
    for (size_t i = 0; i < n_in; i++) {
        REQUIRE(in[i] && in[i]->ncomp == 2, "inputs must be 2-component ciphertexts");
        if (in[i]->level != in[0]->level) throw Error(VR_ELEVEL, "inputs at different levels");
        if (in[i]->scale != in[0]->scale) throw Error(VR_ESCALE, "inputs at different scales");
        r->bufs.push_back(in[i]->buf);
        r->data.push_back(in[i]->data);
    }
    r->level = in[0]->level;
    r->scale = in[0]->scale;
    if (r->level < m.levels()) throw Error(VR_ELEVEL, "not enough levels for the model");
    r->bytes = request_bytes(srv->ctx, m, r->level);
    if (srv->resident > srv->budget || r->bytes > srv->budget - srv->resident)
        throw Error(VR_EBUSY, "request can never fit the memory budget");
    r->session = session_id;
    r->model = model_id;
    r->images = n_images;
    r->ticket = srv->next_ticket++;
    VR_HIP(hipEventCreateWithFlags(&r->ready, hipEventDisableTiming));
    VR_HIP(hipEventRecord(r->ready, srv->ctx->stream));
    r->t_submit = now_ms();
    *ticket = r->ticket;
    srv->pending.push_back(r.get());
    srv->reqs[r->ticket] = std::move(r);
    lk.unlock();
    srv->cv.notify_all();
    API_END
}

vr_status vr_srv_cancel(vr_server* srv, uint64_t ticket)
{
    API_BEGIN
    REQUIRE(srv, "null server");
    std::lock_guard<std::mutex> g(srv->mu);
    auto it = std::find_if(srv->pending.begin(), srv->pending.end(),
                           [ticket](const Request* r) { return r->ticket == ticket; });
    REQUIRE(it != srv->pending.end(), "request is not pending");
    Request* r = *it;
    srv->pending.erase(it);
    r->state = 3;
    r->err = VR_ECANCELED;
    r->msg = "cancelled";
    r->bufs.clear();
    r->data.clear();
    (void)hipEventDestroy(r->ready);
    r->ready = nullptr;
    srv->done_cv.notify_all();
    API_END
}

vr_status vr_srv_poll(vr_server* srv, uint64_t ticket, int wait, vr_ciphertext** out, size_t cap,
                      size_t* n_out, int* ready)
{
    if (n_out) *n_out = 0;
    if (ready) *ready = 0;
    API_BEGIN
    REQUIRE(srv && n_out && ready, "null argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    REQUIRE(it != srv->reqs.end(), "unknown or already collected ticket");
    Request* r = it->second.get();
    if (wait)
        srv->done_cv.wait(lk, [r] { return r->state >= 2; });
    if (r->state < 2) return VR_OK;
    if (r->state == 3) {
        vr_status code = r->err;
        std::string msg = r->msg;
        srv->reqs.erase(it);
        throw Error(code, "request failed: " + msg);
    }
    REQUIRE(out && cap >= r->out.n, "output capacity too small");
    to_handles(srv->ctx, r->out, out);
    *n_out = r->out.n;
    *ready = 1;
    srv->reqs.erase(it);
    API_END
}

vr_status vr_srv_reset_stats(vr_server* srv)
{
    API_BEGIN
    REQUIRE(srv, "null server");
    std::lock_guard<std::mutex> g(srv->mu);
    srv->lat_ms.clear();
    srv->images_done = 0;
    srv->t_first = -1;
    srv->t_last = 0;
    srv->waves = 0;
    srv->batched_requests = 0;
    API_END
}

vr_status vr_srv_stats(vr_server* srv, double* p50_ms, double* p99_ms, double* images_per_s,
                       uint64_t* completed, uint64_t* waves, uint64_t* batched)
{
    API_BEGIN
    REQUIRE(srv, "null server");
    std::lock_guard<std::mutex> g(srv->mu);
    std::vector<double> l = srv->lat_ms;
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {   // nearest rank
        if (l.empty()) return 0.0;
        size_t r = (size_t)std::ceil(p / 100.0 * l.size());
        return l[std::min(l.size(), std::max<size_t>(r, 1)) - 1];
    };
    if (p50_ms) *p50_ms = pct(50);
    if (p99_ms) *p99_ms = pct(99);
    double span = srv->t_last - srv->t_first;
    if (images_per_s) *images_per_s = span > 0 ? srv->images_done / (span / 1e3) : 0.0;
    if (completed) *completed = l.size();
    if (waves) *waves = srv->waves;
    if (batched) *batched = srv->batched_requests;
    API_END
}

}  // extern "C"
