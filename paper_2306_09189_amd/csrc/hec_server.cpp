// hec_server.cpp -- a request loop for encrypted inference (include/hecnn.h,
// "serving").
//
// The paper's threat model (Background): the client encrypts its image and
// decrypts the result; the server evaluates the network with the weights in
// the clear.  A server here holds the evaluation and rotation keys and the
// layer plans resident in HBM and evaluates requests as they arrive:
//
//   * lanes: each lane is a worker thread with its own HIP stream and memory
//     pool over the shared tables and keys, so the work of requests on
//     different lanes overlaps on the device;
//   * admission by memory: every model has a device-memory footprint (the
//     peak of its evaluation, measured when it is registered); requests are
//     taken from the queue in arrival order while the footprints of the
//     requests on the device stay within the budget; a request whose
//     footprint alone exceeds the budget is rejected (HEC_ENOMEM);
//   * continuous batching: when a lane frees up it takes the oldest waiting
//     request together with the later waiting requests of the same model (up
//     to max_batch, as memory allows) and evaluates them as one batch -- in
//     plan mode 4 the rotations of all their shards share each key read.
// Results do not depend on batching: each request's ciphertexts are those of
// evaluating it alone.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

#include "hec_internal.h"

namespace {
typedef std::chrono::steady_clock clk;

struct Model {
    const hec_conv_plan *plan = nullptr;
    int pool_mode = -1;   // -1: no pooling after the convolution
    size_t footprint = 0;  // device bytes of one evaluation (peak, measured)
};

struct Request {
    uint64_t id = 0;
    uint32_t model = 0;
    const hec_image *in = nullptr;
    clk::time_point t_submit, t_start, t_done;
    hec_image *out = nullptr;
    hec_status status = HEC_OK;
    std::string err;
    int state = 0;  // 0 queued, 1 on a lane, 2 done
    uint32_t batch = 0;
};
}  // namespace

struct hec_server {
    hec_ctx *ctx = nullptr;
    hec_server_params prm{};
    std::vector<hec_ctx *> lanes;
    std::vector<std::thread> workers;
    std::vector<Model> models;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    size_t in_use = 0, peak_in_use = 0;
    bool stopping = false, started = false;
    uint64_t next_id = 1;
    // statistics over completed requests
    std::vector<double> lat_ms;
    uint64_t completed = 0, rejected = 0, batches = 0, batched_requests = 0, max_concurrent = 0, running = 0;
    clk::time_point t_first, t_last;
    bool have_first = false;
};

// one evaluation of a model on a lane for several inputs (same model)
static hec_status eval_batch(hec_ctx *lane, const Model &m, const std::vector<const hec_image *> &ins,
                             std::vector<hec_image *> &outs)
{
    std::vector<hec_image *> conv;
    HEC_CHECK(conv_plan_run_multi(lane, m.plan, ins, conv));
    if (m.pool_mode < 0) {
        outs = conv;
        return HEC_OK;
    }
    std::vector<const hec_image *> cin(conv.begin(), conv.end());
    hec_status s = avgpool_multi(lane, cin, m.pool_mode, outs);
    for (auto *im : conv) hec_image_free(im);
    return s;
}

static void worker(hec_server *S, size_t li)
{
    hec_ctx *lane = S->lanes[li];
    hipSetDevice(lane->dev);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // the oldest request decides the model; reject what can never fit
        S->cv_work.wait(lk, [&] {
            if (S->queue.empty()) return S->stopping;
            const Request &h = *S->reqs[S->queue.front()];
            const size_t fp = S->models[h.model].footprint;
            return fp > S->prm.mem_budget || S->in_use + fp <= S->prm.mem_budget;
        });
        if (S->queue.empty()) break;  // stopping and drained
        Request &h = *S->reqs[S->queue.front()];
        const Model &m = S->models[h.model];
        if (m.footprint > S->prm.mem_budget) {
            h.status = HEC_ENOMEM;
            h.err = "request needs more device memory than the server's budget";
            h.state = 2;
            h.t_done = clk::now();
            S->queue.pop_front();
            S->rejected++;
            S->cv_done.notify_all();
            continue;
        }
        // the batch: the head and later waiting requests of its model, in order, as memory allows
        std::vector<Request *> b;
        const uint32_t mid = h.model;
        for (auto it = S->queue.begin(); it != S->queue.end() && b.size() < std::max(1u, S->prm.max_batch);) {
            Request &r = *S->reqs[*it];
            if (r.model == mid && S->in_use + (b.size() + 1) * m.footprint <= S->prm.mem_budget) {
                b.push_back(&r);
                it = S->queue.erase(it);
            } else {
                ++it;
            }
        }
        const size_t need = b.size() * m.footprint;
        S->in_use += need;
        S->peak_in_use = std::max(S->peak_in_use, S->in_use);
        S->running += b.size();
        S->max_concurrent = std::max(S->max_concurrent, S->running);
        S->batches++;
        S->batched_requests += b.size();
        std::vector<const hec_image *> ins;
        for (Request *r : b) {
            r->state = 1;
            r->t_start = clk::now();
            r->batch = (uint32_t)b.size();
            ins.push_back(r->in);
        }
        lk.unlock();
        std::vector<hec_image *> outs;
        hec_status s = eval_batch(lane, m, ins, outs);
        std::string err = s == HEC_OK ? std::string() : std::string(hec_last_error());
        if (s == HEC_OK && hipStreamSynchronize(lane->st) != hipSuccess) {
            s = HEC_EDEVICE;
            err = "lane stream";
        }
        lk.lock();
        const auto now = clk::now();
        for (size_t i = 0; i < b.size(); i++) {
            Request *r = b[i];
            r->status = s;
            r->err = err;
            r->out = s == HEC_OK ? outs[i] : nullptr;
            r->state = 2;
            r->t_done = now;
            if (s == HEC_OK) {
                S->completed++;
                S->lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
                S->t_last = now;
            }
        }
        if (s != HEC_OK)
            for (auto *im : outs) hec_image_free(im);
        S->in_use -= need;
        S->running -= b.size();
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
}

extern "C" hec_status hec_server_start(hec_ctx *c, const hec_server_params *prm, hec_server **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !prm) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (prm->lanes < 1 || prm->lanes > 16) HEC_FAIL(HEC_EINVAL, "1 to 16 lanes");
    if (!prm->mem_budget) HEC_FAIL(HEC_EINVAL, "memory budget must be positive");
    if (!c->have_keys) HEC_FAIL(HEC_ENOKEY, "no keys (call ckks_keygen and generate the rotation keys first)");
    std::unique_ptr<hec_server> S(new hec_server());
    S->ctx = c;
    S->prm = *prm;
    for (uint32_t i = 0; i < prm->lanes; i++) {
        hec_ctx *l = nullptr;
        hec_status s = ctx_lane_create(c, &l);
        if (s != HEC_OK) {
            for (auto *x : S->lanes) ctx_lane_destroy(x);
            return s;
        }
        S->lanes.push_back(l);
    }
    *out = S.release();
    return HEC_OK;
}

extern "C" hec_status hec_server_add_model(hec_server *S, const hec_conv_plan *plan, int pool_mode,
                                           const hec_image *like, uint32_t *model)
{
    if (!S || !plan || !like) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (pool_mode != -1 && pool_mode != 0 && pool_mode != 2 && pool_mode != 3 && pool_mode != 4)
        HEC_FAIL(HEC_EINVAL, "pooling mode must be -1 (none), 0, 2, 3 or 4");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->started) HEC_FAIL(HEC_EBUSY, "models are registered before the first request");
    }
    Model m;
    m.plan = plan;
    m.pool_mode = pool_mode;
    // one evaluation on every lane: the peak of its memory is the footprint,
    // and each lane's caches (pooling masks) are filled before requests come
    for (hec_ctx *l : S->lanes) {
        HEC_CHECK(hec_ctx_sync(S->ctx));
        const size_t before = l->pool.live();
        {
            std::lock_guard<std::mutex> g(l->pool.mu_);
            l->pool.peak_live = l->pool.bytes_live;
        }
        std::vector<hec_image *> outs;
        HEC_CHECK(eval_batch(l, m, {like}, outs));
        HEC_TRY_HIP(hipStreamSynchronize(l->st));
        size_t peak;
        {
            std::lock_guard<std::mutex> g(l->pool.mu_);
            peak = l->pool.peak_live;
        }
        for (auto *im : outs) hec_image_free(im);
        m.footprint = std::max(m.footprint, peak - before);
    }
    std::lock_guard<std::mutex> lk(S->mu);
    S->models.push_back(m);
    if (model) *model = (uint32_t)(S->models.size() - 1);
    return HEC_OK;
}

extern "C" size_t hec_server_model_footprint(const hec_server *S, uint32_t model)
{
    if (!S || model >= S->models.size()) return 0;
    return S->models[model].footprint;
}

static void ensure_started(hec_server *S)
{
    if (S->started) return;
    S->started = true;
    for (size_t i = 0; i < S->lanes.size(); i++) S->workers.emplace_back(worker, S, i);
}

extern "C" hec_status hec_server_submit(hec_server *S, uint32_t model, const hec_image *in, uint64_t *id)
{
    if (!S || !in || !id) HEC_FAIL(HEC_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) HEC_FAIL(HEC_EBUSY, "server is stopping");
    if (model >= S->models.size()) HEC_FAIL(HEC_EINVAL, "no model %u", model);
    ensure_started(S);
    std::unique_ptr<Request> r(new Request());
    r->id = S->next_id++;
    r->model = model;
    r->in = in;
    r->t_submit = clk::now();
    if (!S->have_first) {
        S->t_first = r->t_submit;
        S->have_first = true;
    }
    *id = r->id;
    S->queue.push_back(r->id);
    S->reqs[r->id] = std::move(r);
    S->cv_work.notify_one();
    return HEC_OK;
}

extern "C" hec_status hec_server_poll(hec_server *S, uint64_t id, int wait, hec_image **out, double *latency_ms)
{
    if (!S || !out) HEC_FAIL(HEC_EINVAL, "NULL argument");
    *out = nullptr;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) HEC_FAIL(HEC_EINVAL, "unknown request %llu", (unsigned long long)id);
    if (wait) S->cv_done.wait(lk, [&] { return it->second->state == 2; });
    Request &r = *it->second;
    if (r.state != 2) HEC_FAIL(HEC_EBUSY, "request %llu not done", (unsigned long long)id);
    hec_status s = r.status;
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
    if (s == HEC_OK) *out = r.out;
    else hec_set_error("%s", r.err.c_str());
    S->reqs.erase(it);
    return s;
}

extern "C" hec_status hec_server_stats(hec_server *S, hec_server_stats_t *st)
{
    if (!S || !st) HEC_FAIL(HEC_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    memset(st, 0, sizeof(*st));
    st->completed = S->completed;
    st->rejected = S->rejected;
    st->batches = S->batches;
    st->batched_requests = S->batched_requests;
    st->max_concurrent = S->max_concurrent;
    st->peak_mem = S->peak_in_use;
    std::vector<double> v = S->lat_ms;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto q = [&](double p) { return v[std::min(v.size() - 1, (size_t)(p * (v.size() - 1) + 0.5))]; };
        st->p50_ms = q(0.50);
        st->p99_ms = q(0.99);
        double sum = 0;
        for (double x : v) sum += x;
        st->mean_ms = sum / v.size();
        const double span = std::chrono::duration<double>(S->t_last - S->t_first).count();
        st->req_per_s = span > 0 ? v.size() / span : 0;
    }
    return HEC_OK;
}

extern "C" hec_status hec_server_stop(hec_server *S)
{
    if (!S) HEC_FAIL(HEC_EINVAL, "NULL argument");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    for (auto &t : S->workers) t.join();
    // results never polled go with the server
    for (auto &kv : S->reqs)
        if (kv.second->out) hec_image_free(kv.second->out);
    for (auto *l : S->lanes) ctx_lane_destroy(l);
    delete S;
    return HEC_OK;
}
