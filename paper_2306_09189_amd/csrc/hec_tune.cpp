// hec_tune.cpp -- launch parameters and the autotuner that picks them
// (include/hecnn.h, "tuning").
//
// The parameters (TuneParams) change how work is cut into launches -- the
// 2^16 NTT's radix and tile, how many limbs one transform launch takes, how
// many rotations or amounts share a key-switch launch -- never the residues.
// The autotuner times a convolution plan on a given input under each
// candidate value, one parameter after the other (coordinate descent from the
// current values), keeps a candidate only if the plan's output is the same
// bit for bit as under the starting values and it is faster, and leaves the
// best values set.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>

#include "hec_internal.h"

namespace {
struct Tunable {
    const char *name;
    int TuneParams::*field;
    std::vector<int> candidates;
};
const std::vector<Tunable> &tunables()
{
    static const std::vector<Tunable> t = {
        {"ntt16_radix", &TuneParams::ntt16_radix, {16, 2}},
        {"ntt_fp64", &TuneParams::ntt_fp64, {1, 0}},
        {"ntt_row_vals", &TuneParams::ntt_row_vals, {16, 8}},
        {"ntt_tile", &TuneParams::ntt_tile, {2048, 4096, 8192}},
        {"ntt_group", &TuneParams::ntt_group, {0, 64, 256, 1024}},
        {"ks_rot_batch", &TuneParams::ks_rot_batch, {4, 8, 16, 32}},
        {"ks_overlap", &TuneParams::ks_overlap, {0, 1}},
        {"ks_amounts", &TuneParams::ks_amounts, {1, 2, 4, 8, 16}},
    };
    return t;
}
const Tunable *find(const char *name)
{
    for (auto &t : tunables())
        if (name && !strcmp(t.name, name)) return &t;
    return nullptr;
}

// the plan's output shards, as stored on the device, copied to the host
hec_status snapshot(hec_ctx *c, const hec_image *img, std::vector<u64> &h)
{
    h.clear();
    for (auto *ct : img->shards) {
        const size_t w = 2ull * (ct->level + 1) * c->n, o = h.size();
        h.resize(o + w);
        HEC_TRY_HIP(hipMemcpyAsync(h.data() + o, ct->d, w * 8, hipMemcpyDeviceToHost, c->st));
    }
    HEC_TRY_HIP(hipStreamSynchronize(c->st));
    return HEC_OK;
}

// median time of `reps` plan runs (after one untimed run whose output is
// compared with ref, when given); *same = output equals ref
hec_status time_runs(hec_ctx *c, const hec_conv_plan *p, const hec_image *in, uint32_t reps,
                     const std::vector<u64> *ref, bool *same, double *ms)
{
    hec_image *out = nullptr;
    HEC_CHECK(he_conv2d_plan_run(c, p, in, &out));
    std::vector<u64> h;
    hec_status s = snapshot(c, out, h);
    hec_image_free(out);
    HEC_CHECK(s);
    if (same) *same = !ref || h == *ref;
    hipEvent_t e0, e1;
    HEC_TRY_HIP(hipEventCreate(&e0));
    HEC_TRY_HIP(hipEventCreate(&e1));
    std::vector<double> t;
    for (uint32_t r = 0; r < reps && s == HEC_OK; r++) {
        hipEventRecord(e0, c->st);
        s = he_conv2d_plan_run(c, p, in, &out);
        hipEventRecord(e1, c->st);
        if (s != HEC_OK) break;
        float f = 0;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&f, e0, e1) != hipSuccess)
            s = HEC_EDEVICE, hec_set_error("tuning timer");
        hec_image_free(out);
        t.push_back(f);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    HEC_CHECK(s);
    std::sort(t.begin(), t.end());
    *ms = t.empty() ? 0.0 : t[t.size() / 2];
    return HEC_OK;
}
}  // namespace

extern "C" hec_status hec_tune_set(const char *name, int64_t value)
{
    const Tunable *t = find(name);
    if (!t) HEC_FAIL(HEC_EINVAL, "no tunable parameter '%s'", name ? name : "(null)");
    if (std::find(t->candidates.begin(), t->candidates.end(), (int)value) == t->candidates.end())
        HEC_FAIL(HEC_EINVAL, "value %lld not among the candidates of %s", (long long)value, name);
    hec_tune_params().*(t->field) = (int)value;
    return HEC_OK;
}

extern "C" hec_status hec_tune_get(const char *name, int64_t *value)
{
    const Tunable *t = find(name);
    if (!t || !value) HEC_FAIL(HEC_EINVAL, "no tunable parameter '%s'", name ? name : "(null)");
    *value = hec_tune_params().*(t->field);
    return HEC_OK;
}

extern "C" hec_status hec_tune_describe(char *buf, size_t cap)
{
    if (!buf || !cap) HEC_FAIL(HEC_EINVAL, "no buffer");
    std::string s;
    for (auto &t : tunables()) {
        if (!s.empty()) s += " ";
        s += std::string(t.name) + "=" + std::to_string(hec_tune_params().*(t.field));
    }
    if (s.size() + 1 > cap) HEC_FAIL(HEC_EINVAL, "buffer of %zu bytes too small", cap);
    memcpy(buf, s.c_str(), s.size() + 1);
    return HEC_OK;
}

extern "C" hec_status hec_tune_save(const char *path)
{
    if (!path) HEC_FAIL(HEC_EINVAL, "path is NULL");
    FILE *f = fopen(path, "w");
    if (!f) HEC_FAIL(HEC_EINVAL, "cannot write %s", path);
    for (auto &t : tunables()) fprintf(f, "%s %d\n", t.name, hec_tune_params().*(t.field));
    fclose(f);
    return HEC_OK;
}

extern "C" hec_status hec_tune_load(const char *path)
{
    if (!path) HEC_FAIL(HEC_EINVAL, "path is NULL");
    FILE *f = fopen(path, "r");
    if (!f) HEC_FAIL(HEC_EINVAL, "cannot read %s", path);
    char name[64];
    long long v;
    hec_status s = HEC_OK;
    while (s == HEC_OK && fscanf(f, "%63s %lld", name, &v) == 2) s = hec_tune_set(name, v);
    fclose(f);
    return s;
}

extern "C" hec_status hec_autotune_conv(hec_ctx *c, const hec_conv_plan *plan, const hec_image *in, uint32_t reps,
                                        char *report, size_t cap)
{
    if (!c || !plan || !in) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (reps < 1) reps = 1;
    HEC_TRY_HIP(hipSetDevice(c->dev));
    TuneParams &tp = hec_tune_params();
    // the reference output and time under the starting values
    std::vector<u64> ref;
    {
        hec_image *out = nullptr;
        HEC_CHECK(he_conv2d_plan_run(c, plan, in, &out));
        hec_status s = snapshot(c, out, ref);
        hec_image_free(out);
        HEC_CHECK(s);
    }
    double best = 0;
    bool same = true;
    HEC_CHECK(time_runs(c, plan, in, reps, nullptr, nullptr, &best));
    std::string log = "start " + std::to_string(best) + " ms;";
    for (auto &t : tunables()) {
        const int keep = tp.*(t.field);
        int chosen = keep;
        for (int v : t.candidates) {
            if (v == keep) continue;
            tp.*(t.field) = v;
            double ms = 0;
            hec_status s = time_runs(c, plan, in, reps, &ref, &same, &ms);
            if (s != HEC_OK) {
                tp.*(t.field) = keep;
                return s;
            }
            char line[96];
            snprintf(line, sizeof(line), " %s=%d %.3f ms%s", t.name, v, ms, same ? "" : " (output differs: rejected)");
            log += line;
            // a candidate must give the same bits and beat the best by more than the timing noise
            if (same && ms < best * 0.98) {
                best = ms;
                chosen = v;
            }
        }
        tp.*(t.field) = chosen;
        log += ";";
    }
    char cfg[256];
    hec_tune_describe(cfg, sizeof(cfg));
    log = std::string("chosen ") + cfg + " " + std::to_string(best) + " ms; " + log;
    if (report && cap) {
        const size_t m = std::min(cap - 1, log.size());
        memcpy(report, log.data(), m);
        report[m] = 0;
    }
    return HEC_OK;
}
