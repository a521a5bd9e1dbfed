// hec_block.cpp -- the repeated unit of the encrypted ResNets: convolution
// with batch norm folded into its weights and bias (Section 4.3, Batch
// Normalization), GELU as a Chebyshev series (Section 4.3, GELU), a second
// convolution with its batch norm folded, and 2x2 average pooling (Section
// 4.2).  The map of the activation's interval [-bound, bound] onto [-1, 1] is
// folded into the first convolution as well, so the series is evaluated on
// [-1, 1] without a level of its own.
#include <cmath>
#include <memory>
#include <set>

#include "hec_internal.h"

struct hec_block {
    hec_ctx *ctx = nullptr;
    Layout in;
    uint32_t level = 0, act_level = 0;
    int mode = 0;
    hec_conv_plan *p1 = nullptr, *p2 = nullptr;
    std::vector<double> b1, b2;
    bool has_b2 = false;
    std::vector<double> coeffs;
    std::set<int32_t> steps;
};

extern "C" void he_block_free(hec_block *b)
{
    if (!b) return;
    he_conv2d_plan_free(b->p1);
    he_conv2d_plan_free(b->p2);
    delete b;
}

// w' = w[o] * (gamma[o] / div), b' = shift[o] / div (every product one IEEE operation)
static void fold(const double *w, size_t per_out, uint32_t Co, const double *gamma, const double *shift, double div,
                 std::vector<double> &wf, std::vector<double> &bf)
{
    wf.resize(per_out * Co);
    bf.resize(Co);
    for (uint32_t o = 0; o < Co; o++) {
        const double s = gamma[o] / div;
        for (size_t i = 0; i < per_out; i++) wf[o * per_out + i] = w[o * per_out + i] * s;
        bf[o] = shift[o] / div;
    }
}

extern "C" hec_status he_block_create(hec_ctx *c, const hec_image *like, const double *w1, uint32_t C1,
                                      const double *bn1, const double *w2, uint32_t C2, const double *bn2, uint32_t k,
                                      double bound, const double *coeffs, size_t ncoeffs, int mode, hec_block **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !like || !w1 || !bn1 || !w2 || !coeffs) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (!C1 || !C2 || k == 0 || k % 2 == 0) HEC_FAIL(HEC_EINVAL, "channels must be positive and the kernel odd");
    if (!(bound > 0.0) || !std::isfinite(bound)) HEC_FAIL(HEC_EINVAL, "the activation bound must be positive");
    if (mode < 0 || mode > 3) HEC_FAIL(HEC_EINVAL, "mode must be 0..3");
    if (like->shards.empty()) HEC_FAIL(HEC_ELAYOUT, "empty image");
    const uint32_t lvl = like->shards[0]->level;
    for (auto *s : like->shards)
        if (s->level != lvl) HEC_FAIL(HEC_ELEVEL, "shards at different levels");
    if (lvl < 2) HEC_FAIL(HEC_ELEVEL, "too few levels for the block");
    for (uint32_t o = 0; o < C1; o++)
        if (!std::isfinite(bn1[o]) || !std::isfinite(bn1[C1 + o])) HEC_FAIL(HEC_EINVAL, "batch norm not finite");
    if (bn2)
        for (uint32_t o = 0; o < C2; o++)
            if (!std::isfinite(bn2[o]) || !std::isfinite(bn2[C2 + o])) HEC_FAIL(HEC_EINVAL, "batch norm not finite");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    std::unique_ptr<hec_block, void (*)(hec_block *)> b(new hec_block(), he_block_free);
    b->ctx = c;
    b->in = like->lay;
    b->level = lvl;
    b->mode = mode;
    b->coeffs.assign(coeffs, coeffs + ncoeffs);
    const uint32_t C = like->lay.C;
    std::vector<double> w1f, w2f;
    fold(w1, (size_t)C * k * k, C1, bn1, bn1 + C1, bound, w1f, b->b1);
    HEC_CHECK(conv_plan_create(c, like->lay, lvl, w1f.data(), C1, k, k, 1, k / 2, &b->p1));
    HEC_CHECK(he_conv2d_plan_set_mode(b->p1, mode));
    // the activation's output level, from a run over levels only
    HEC_CHECK(cheb_levels(c, lvl - 1, like->shards[0]->scale, coeffs, ncoeffs, -1.0, 1.0, &b->act_level, nullptr));
    if (b->act_level < 1) HEC_FAIL(HEC_ELEVEL, "too few levels after the activation");
    if (bn2) {
        fold(w2, (size_t)C1 * k * k, C2, bn2, bn2 + C2, 1.0, w2f, b->b2);
        b->has_b2 = true;
    } else {
        w2f.assign(w2, w2 + (size_t)C2 * C1 * k * k);
    }
    HEC_CHECK(conv_plan_create(c, conv_plan_out(b->p1), b->act_level, w2f.data(), C2, k, k, 1, k / 2, &b->p2));
    HEC_CHECK(he_conv2d_plan_set_mode(b->p2, mode));
    for (hec_conv_plan *p : {b->p1, b->p2}) {
        size_t n = 0;
        HEC_CHECK(he_conv2d_plan_steps(p, nullptr, 0, &n));
        std::vector<int32_t> st(n);
        HEC_CHECK(he_conv2d_plan_steps(p, st.data(), n, &n));
        b->steps.insert(st.begin(), st.end());
    }
    pool_steps(conv_plan_out(b->p2), false, b->act_level - 1, b->steps);
    *out = b.release();
    return HEC_OK;
}

extern "C" hec_status he_block_steps(const hec_block *b, int32_t *steps, size_t cap, size_t *count)
{
    if (!b) HEC_FAIL(HEC_EINVAL, "block is NULL");
    if (count) *count = b->steps.size();
    if (steps) {
        if (cap < b->steps.size()) HEC_FAIL(HEC_EINVAL, "capacity too small");
        size_t i = 0;
        for (int32_t s : b->steps) steps[i++] = s;
    }
    return HEC_OK;
}

extern "C" hec_status he_block_run(hec_ctx *c, const hec_block *b, const hec_image *in, hec_image **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !b || !in) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (b->ctx != c) HEC_FAIL(HEC_EINVAL, "block of another context");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    auto img = [](hec_image *p) { return std::unique_ptr<hec_image, void (*)(hec_image *)>(p, hec_image_free); };
    hec_image *t = nullptr;
    HEC_CHECK(he_conv2d_plan_run(c, b->p1, in, &t));
    auto x1 = img(t);
    auto x2 = img(new hec_image());
    x2->ctx = c;
    x2->lay = x1->lay;
    HEC_CHECK(image_add_bias(c, x1->shards, x1->lay, b->b1.data(), x2->shards));
    x1.reset();
    auto x3 = img(new hec_image());
    x3->ctx = c;
    x3->lay = x2->lay;
    HEC_CHECK(cheb_image(c, x2->shards, b->coeffs.data(), b->coeffs.size(), -1.0, 1.0, x3->shards));
    x2.reset();
    HEC_CHECK(he_conv2d_plan_run(c, b->p2, x3.get(), &t));
    auto x4 = img(t);
    x3.reset();
    if (b->has_b2) {
        auto x5 = img(new hec_image());
        x5->ctx = c;
        x5->lay = x4->lay;
        HEC_CHECK(image_add_bias(c, x4->shards, x4->lay, b->b2.data(), x5->shards));
        x4 = std::move(x5);
    }
    return he_avgpool_ex(c, x4.get(), 2, b->mode >= 2 ? b->mode : 0, out);
}
