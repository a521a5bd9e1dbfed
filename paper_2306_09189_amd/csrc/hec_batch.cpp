// hec_batch.cpp -- batches of layer evaluations launched as one captured HIP
// graph (include/hecnn.h, "batches").
//
// A batch is a list of (convolution plan, input image) items, typically
// ciphertexts of several images at different levels (and so different limb
// counts).  Eagerly, the items run one after another on the context stream.
// In graph mode the first launch records the items into one HIP graph and
// every launch replays it: the launch cost of the thousands of kernels of a
// batch is paid once, and the graph's memory (its temporaries and its
// outputs) stays with the batch, so a replay rewrites the same outputs from
// the current contents of the same inputs.
#include <cstring>

#include "hec_internal.h"

struct hec_batch {
    hec_ctx *ctx = nullptr;
    struct Item {
        const hec_conv_plan *plan;
        const hec_image *in;
    };
    std::vector<Item> items;
    std::vector<hec_image *> eouts;  // results of the last eager launch (context pool)
    std::vector<hec_image *> gouts;  // the graph's outputs (in gmem, rewritten by every replay)
    bool last_graph = false;         // the last launch replayed the graph
    DevPool gmem;                    // memory the captured graph reads and writes
    hipStream_t cs = nullptr;       // capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void free_images(hec_batch *b, std::vector<hec_image *> &v, bool graph_memory)
{
    if (graph_memory) {
        // graph-owned memory goes back to the batch, which releases it at the end
        PoolScope ps(b->ctx, &b->gmem);
        for (auto *im : v) hec_image_free(im);
    } else {
        for (auto *im : v) hec_image_free(im);
    }
    v.clear();
}

// run every item on the context's current stream and pool; results into outs
static hec_status run_items(hec_batch *b, std::vector<hec_image *> &outs)
{
    outs.assign(b->items.size(), nullptr);
    for (size_t i = 0; i < b->items.size(); i++) {
        hec_status s = he_conv2d_plan_run(b->ctx, b->items[i].plan, b->items[i].in, &outs[i]);
        if (s != HEC_OK) {
            for (auto *im : outs) hec_image_free(im);
            outs.clear();
            return s;
        }
    }
    return HEC_OK;
}

extern "C" hec_status hec_batch_begin(hec_ctx *c, hec_batch **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c) HEC_FAIL(HEC_EINVAL, "ctx is NULL");
    hec_batch *b = new hec_batch();
    b->ctx = c;
    b->gmem.trimmable = false;
    *out = b;
    return HEC_OK;
}

extern "C" hec_status hec_batch_add(hec_batch *b, const hec_conv_plan *plan, const hec_image *in, uint32_t *index)
{
    if (!b || !plan || !in) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (b->exec) HEC_FAIL(HEC_EBUSY, "the batch has been captured; items cannot be added");
    b->items.push_back({plan, in});
    if (index) *index = (uint32_t)(b->items.size() - 1);
    return HEC_OK;
}

static hec_status capture(hec_batch *b)
{
    hec_ctx *c = b->ctx;
    // one eager run on the batch's memory first: the recorded run then finds
    // every block it asks for cached, so nothing is allocated while recording
    {
        PoolScope ps(c, &b->gmem);
        std::vector<hec_image *> warm;
        HEC_CHECK(run_items(b, warm));
        for (auto *im : warm) hec_image_free(im);
    }
    HEC_TRY_HIP(hipStreamSynchronize(c->st));
    if (!b->cs) HEC_TRY_HIP(hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking));
    hipStream_t prev = c->st;
    c->st = b->cs;
    std::vector<hec_image *> outs;
    hec_status s = HEC_OK;
    {
        PoolScope ps(c, &b->gmem);
        hipError_t e = hipStreamBeginCapture(b->cs, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) {
            c->st = prev;
            HEC_FAIL(HEC_EDEVICE, "stream capture: %s", hipGetErrorString(e));
        }
        s = run_items(b, outs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cs, &g);
        if (s == HEC_OK && e != hipSuccess) s = HEC_EDEVICE, hec_set_error("stream capture: %s", hipGetErrorString(e));
        if (s == HEC_OK) {
            b->graph = g;
            e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                b->exec = nullptr;
                s = HEC_EDEVICE;
                hec_set_error("graph instantiation: %s", hipGetErrorString(e));
            }
        } else if (g) {
            hipGraphDestroy(g);
        }
        if (s != HEC_OK)
            for (auto *im : outs) hec_image_free(im);
    }
    c->st = prev;
    if (s != HEC_OK) return s;
    b->gouts = outs;
    return HEC_OK;
}

extern "C" hec_status hec_batch_launch(hec_batch *b, int mode)
{
    if (!b) HEC_FAIL(HEC_EINVAL, "batch is NULL");
    hec_ctx *c = b->ctx;
    HEC_TRY_HIP(hipSetDevice(c->dev));
    if (mode == HEC_BATCH_EAGER) {
        std::vector<hec_image *> outs;
        HEC_CHECK(run_items(b, outs));
        free_images(b, b->eouts, false);
        b->eouts = outs;
        b->last_graph = false;
        return HEC_OK;
    }
    if (mode != HEC_BATCH_GRAPH) HEC_FAIL(HEC_EINVAL, "batch mode must be HEC_BATCH_EAGER or HEC_BATCH_GRAPH");
    if (!b->exec) HEC_CHECK(capture(b));
    HEC_TRY_HIP(hipGraphLaunch(b->exec, c->st));
    b->last_graph = true;
    return HEC_OK;
}

extern "C" const hec_image *hec_batch_output(const hec_batch *b, uint32_t i)
{
    if (!b) return nullptr;
    const auto &v = b->last_graph ? b->gouts : b->eouts;
    return i < v.size() ? v[i] : nullptr;
}

extern "C" uint32_t hec_batch_size(const hec_batch *b) { return b ? (uint32_t)b->items.size() : 0; }

extern "C" void hec_batch_free(hec_batch *b)
{
    if (!b) return;
    hipSetDevice(b->ctx->dev);
    hipStreamSynchronize(b->ctx->st);
    free_images(b, b->eouts, false);
    free_images(b, b->gouts, true);
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->cs) hipStreamDestroy(b->cs);
    b->gmem.release_all();
    delete b;
}
