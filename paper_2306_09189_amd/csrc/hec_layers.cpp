// hec_layers.cpp -- image packing, homomorphic conv2d and 2x2 average pooling
// (Section 4 of the paper) on top of the ciphertext operations.
//
// Layout: each channel is a row-major block of B = mp*mp slots (mp = side
// padded to a power of two); a shard is a ciphertext of N/B blocks with a
// block map lam[b] = logical channel of block b (-1 = empty).  Duplication
// (consecutive d-fold copies) and the permutation left by consolidation are
// both block maps, so a convolution reads K^{lam(b+r), mu(b)} wherever the
// paper reads K^{tau(i)}.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>
#include <sstream>

#include "hec_internal.h"

hec_status decrypt_slots(hec_ctx *c, const hec_ct *ct, double *z, size_t nz);

static uint32_t next_pow2(uint32_t x)
{
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

Layout natural_layout(uint32_t N, uint32_t C, uint32_t H, uint32_t W, uint32_t mp)
{
    Layout L;
    L.N = N; L.C = C; L.H = H; L.W = W;
    L.mp = mp ? mp : next_pow2(std::max(H, W));
    const uint32_t B = L.B();
    if (B > N) {
        // channel shards: each channel split into consecutive-row shards
        L.channel = true;
        for (uint32_t f = 0; f < C; f++)
            for (uint32_t v = 0; v < B / N; v++) L.cs.push_back({(int32_t)f, (int32_t)v});
        return L;
    }
    const uint32_t nb = N / B, Cp = next_pow2(C);
    if ((uint64_t)Cp * B <= N) {
        uint32_t d = N / (Cp * B);
        std::vector<int32_t> m(nb);
        for (uint32_t b = 0; b < nb; b++) m[b] = (b / d < C) ? (int32_t)(b / d) : -1;
        L.maps.push_back(m);
    } else {
        uint32_t t = (C + nb - 1) / nb;  // no shard is left entirely empty
        for (uint32_t u = 0; u < t; u++) {
            std::vector<int32_t> m(nb);
            for (uint32_t b = 0; b < nb; b++) m[b] = (u * nb + b < C) ? (int32_t)(u * nb + b) : -1;
            L.maps.push_back(m);
        }
    }
    return L;
}

static void pack_shard(const Layout &L, const double *x, uint32_t u, std::vector<double> &v)
{
    const uint32_t B = L.B();
    v.assign(L.N, 0.0);
    if (L.channel) {
        const int32_t f = L.cs[u].first, part = L.cs[u].second;
        const uint32_t R = L.R();
        for (uint32_t r = 0; r < R; r++) {
            uint32_t i = part * R + r;
            if (i >= L.H) break;
            for (uint32_t j = 0; j < L.W; j++) v[(size_t)r * L.mp + j] = x[((size_t)f * L.H + i) * L.W + j];
        }
        return;
    }
    for (uint32_t b = 0; b < L.nb(); b++) {
        int32_t f = L.maps[u][b];
        if (f < 0) continue;
        for (uint32_t i = 0; i < L.H; i++)
            for (uint32_t j = 0; j < L.W; j++) v[(size_t)b * B + i * L.mp + j] = x[((size_t)f * L.H + i) * L.W + j];
    }
}

static hec_image *image_new(hec_ctx *c, const Layout &L)
{
    hec_image *im = new hec_image();
    im->ctx = c;
    im->lay = L;
    return im;
}

extern "C" void hec_image_free(hec_image *img)
{
    if (!img) return;
    for (auto *s : img->shards) ct_free(s);
    delete img;
}

extern "C" hec_status he_image_encrypt(hec_ctx *c, const double *x, uint32_t C, uint32_t H, uint32_t W, uint32_t level,
                                       uint64_t seed, hec_image **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !x || !C || !H || !W) HEC_FAIL(HEC_EINVAL, "bad image arguments");
    if (level > c->L) HEC_FAIL(HEC_ELEVEL, "level above L");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    Layout L = natural_layout(c->N, C, H, W);
    if (!L.shards()) HEC_FAIL(HEC_ELAYOUT, "empty layout");
    std::vector<std::vector<double>> v(L.shards());
    std::vector<const double *> zp;
    for (uint32_t u = 0; u < L.shards(); u++) {
        pack_shard(L, x, u, v[u]);
        zp.push_back(v[u].data());
    }
    std::vector<hec_pt *> pts;
    HEC_CHECK(pt_encode_many(c, zp, c->N, level, std::ldexp(1.0, (int)c->prm.log_scale), pts));
    hec_image *im = image_new(c, L);
    for (uint32_t u = 0; u < pts.size(); u++) {
        hec_ct *ct = nullptr;
        hec_status s = ckks_encrypt_idx(c, pts[u], seed, u, &ct);
        if (s != HEC_OK) {
            for (auto *p : pts) pt_free(p);
            hec_image_free(im);
            return s;
        }
        im->shards.push_back(ct);
    }
    for (auto *p : pts) pt_free(p);
    *out = im;
    return HEC_OK;
}

extern "C" hec_status he_image_decrypt(hec_ctx *c, const hec_image *img, double *x)
{
    if (!c || !img || !x) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    const Layout &L = img->lay;
    std::vector<char> seen(L.C, 0);
    std::vector<double> z(c->N);
    if (L.channel) {
        const uint32_t R = L.R();
        for (uint32_t u = 0; u < L.cs.size(); u++) {
            const int32_t f = L.cs[u].first, part = L.cs[u].second;
            if ((uint32_t)part * R >= L.H) continue;
            HEC_CHECK(decrypt_slots(c, img->shards[u], z.data(), c->N));
            for (uint32_t r = 0; r < R && part * R + r < L.H; r++)
                for (uint32_t j = 0; j < L.W; j++)
                    x[((size_t)f * L.H + part * R + r) * L.W + j] = z[(size_t)r * L.mp + j];
            seen[f] = 1;
        }
    }
    for (uint32_t u = 0; u < L.maps.size(); u++) {
        bool need = false;
        for (int32_t f : L.maps[u]) need |= (f >= 0 && !seen[f]);
        if (!need) continue;
        HEC_CHECK(decrypt_slots(c, img->shards[u], z.data(), c->N));
        for (uint32_t b = 0; b < L.nb(); b++) {
            int32_t f = L.maps[u][b];
            if (f < 0 || seen[f]) continue;
            seen[f] = 1;
            for (uint32_t i = 0; i < L.H; i++)
                for (uint32_t j = 0; j < L.W; j++)
                    x[((size_t)f * L.H + i) * L.W + j] = z[(size_t)b * L.B() + i * L.mp + j];
        }
    }
    for (uint32_t f = 0; f < L.C; f++)
        if (!seen[f]) HEC_FAIL(HEC_ELAYOUT, "channel %u is not present in the image", f);
    return HEC_OK;
}

extern "C" hec_status he_image_info(const hec_image *img, uint32_t *C, uint32_t *H, uint32_t *W, uint32_t *mp,
                                    uint32_t *n_shards)
{
    if (!img) HEC_FAIL(HEC_EINVAL, "img is NULL");
    if (C) *C = img->lay.C;
    if (H) *H = img->lay.H;
    if (W) *W = img->lay.W;
    if (mp) *mp = img->lay.mp;
    if (n_shards) *n_shards = (uint32_t)img->shards.size();
    return HEC_OK;
}

extern "C" hec_status he_image_block_map(const hec_image *img, uint32_t u, int32_t *lam, size_t cap)
{
    if (!img || !lam) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (img->lay.channel) HEC_FAIL(HEC_ELAYOUT, "channel-sharded image: use he_image_channel_shard");
    if (u >= img->lay.maps.size()) HEC_FAIL(HEC_EINVAL, "no shard %u", u);
    if (cap < img->lay.nb()) HEC_FAIL(HEC_EINVAL, "capacity too small");
    memcpy(lam, img->lay.maps[u].data(), img->lay.nb() * 4);
    return HEC_OK;
}

extern "C" hec_status he_image_channel_shard(const hec_image *img, uint32_t u, int32_t *channel, int32_t *part)
{
    if (!img || !channel || !part) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (!img->lay.channel) HEC_FAIL(HEC_ELAYOUT, "image-sharded image: use he_image_block_map");
    if (u >= img->lay.cs.size()) HEC_FAIL(HEC_EINVAL, "no shard %u", u);
    *channel = img->lay.cs[u].first;
    *part = img->lay.cs[u].second;
    return HEC_OK;
}

extern "C" const hec_ct *he_image_shard(const hec_image *img, uint32_t u)
{
    return (img && u < img->shards.size()) ? img->shards[u] : nullptr;
}

// ---------------------------------------------------------------------------
// convolution planning (Section 4.1)
// ---------------------------------------------------------------------------
struct ConvItem {
    int32_t amount;
    int32_t baby, giant;  // amount = baby + giant (mod N): block offset r*B (0 for channel shards), tap offset
    std::vector<std::pair<uint32_t, std::vector<double>>> pts;  // output shard -> slot vector
    // image shards: the tap (kr * kw + kc) and, per entry of pts, its nonzero
    // block weights (block, weight): the slot vector is weight * tap mask per block
    int32_t tap = -1;
    std::vector<std::vector<std::pair<uint32_t, double>>> bw;
};

// Offsets r with, per needed output block b, the input channel lam[b+r] it
// takes: first the offsets that give every needed block a new channel at
// once, then block-by-block completion; smallest offset first.
static bool rotation_offsets(const std::vector<int32_t> &lam, const std::vector<uint32_t> &need_b,
                             std::vector<std::pair<uint32_t, std::map<uint32_t, int32_t>>> &res)
{
    const uint32_t nb = (uint32_t)lam.size();
    std::set<int32_t> chans;
    for (int32_t f : lam)
        if (f >= 0) chans.insert(f);
    std::map<uint32_t, std::set<int32_t>> cov;
    std::map<uint32_t, std::map<uint32_t, int32_t>> assign;
    for (uint32_t r = 0; r < nb; r++) {
        bool all = true;
        for (uint32_t b : need_b) {
            int32_t f = lam[(b + r) % nb];
            if (f < 0 || cov[b].count(f)) { all = false; break; }
        }
        if (!all) continue;
        for (uint32_t b : need_b) {
            int32_t f = lam[(b + r) % nb];
            assign[r][b] = f;
            cov[b].insert(f);
        }
    }
    for (uint32_t r = 0; r < nb; r++)
        for (uint32_t b : need_b) {
            int32_t f = lam[(b + r) % nb];
            if (f >= 0 && !cov[b].count(f)) {
                assign[r][b] = f;
                cov[b].insert(f);
            }
        }
    for (uint32_t b : need_b)
        if (cov[b] != chans) return false;
    res.clear();
    for (auto &kv : assign) res.push_back(kv);
    return true;
}

static void tap_mask(const Layout &L, uint32_t Ho, uint32_t Wo, int dk, int dl, std::vector<double> &m, bool &any)
{
    m.assign(L.B(), 0.0);
    any = false;
    for (int i = 0; i < (int)L.mp; i++)
        for (int j = 0; j < (int)L.mp; j++) {
            bool ok = i < (int)Ho && j < (int)Wo && i + dk >= 0 && i + dk < (int)L.H && j + dl >= 0 &&
                      j + dl < (int)L.W;
            if (ok) {
                m[(size_t)i * L.mp + j] = 1.0;
                any = true;
            }
        }
}

static hec_status conv_items(const Layout &L, const double *w, uint32_t Co, uint32_t kh, uint32_t kw, uint32_t pad,
                             Layout &out, std::vector<std::vector<ConvItem>> &plan)
{
    const int Ho = (int)L.H + 2 * (int)pad - (int)kh + 1, Wo = (int)L.W + 2 * (int)pad - (int)kw + 1;
    if (Ho < 1 || Wo < 1 || Ho > (int)L.mp || Wo > (int)L.mp) HEC_FAIL(HEC_ELAYOUT, "bad convolution geometry");
    out = natural_layout(L.N, Co, Ho, Wo, L.mp);
    if (out.maps.empty()) HEC_FAIL(HEC_ELAYOUT, "output does not fit image shards");
    const uint32_t N = L.N, B = L.B(), nb = L.nb(), Ci = L.C;
    std::vector<uint32_t> need_b;
    for (uint32_t b = 0; b < nb; b++) {
        bool any = false;
        for (auto &mu : out.maps) any |= mu[b] >= 0;
        if (any) need_b.push_back(b);
    }
    plan.assign(L.maps.size(), {});
    std::vector<double> mask;
    for (uint32_t u = 0; u < L.maps.size(); u++) {
        std::vector<std::pair<uint32_t, std::map<uint32_t, int32_t>>> offs;
        if (!rotation_offsets(L.maps[u], need_b, offs)) HEC_FAIL(HEC_ELAYOUT, "layout cannot be convolved");
        for (auto &ro : offs) {
            const uint32_t r = ro.first;
            for (uint32_t kr = 0; kr < kh; kr++)
                for (uint32_t kc = 0; kc < kw; kc++) {
                    int dk = (int)kr - (int)pad, dl = (int)kc - (int)pad;
                    bool any;
                    tap_mask(L, Ho, Wo, dk, dl, mask, any);
                    if (!any) continue;
                    int64_t a = ((int64_t)r * B + (int64_t)dk * L.mp + dl) % (int64_t)N;
                    if (a < 0) a += N;
                    int64_t gi = ((int64_t)dk * L.mp + dl) % (int64_t)N;
                    if (gi < 0) gi += N;
                    ConvItem it;
                    it.amount = (int32_t)a;
                    it.baby = (int32_t)(((int64_t)r * B) % (int64_t)N);
                    it.giant = (int32_t)gi;
                    it.tap = (int32_t)(kr * kw + kc);
                    for (uint32_t v = 0; v < out.maps.size(); v++) {
                        std::vector<double> vec(N, 0.0);
                        std::vector<std::pair<uint32_t, double>> bw;
                        for (auto &bf : ro.second) {
                            int32_t g = out.maps[v][bf.first];
                            if (g < 0) continue;
                            double wv = w[(((size_t)g * Ci + bf.second) * kh + kr) * kw + kc];
                            if (wv == 0.0) continue;
                            double *dst = &vec[(size_t)bf.first * B];
                            for (uint32_t e = 0; e < B; e++) dst[e] = wv * mask[e];
                            bw.push_back({bf.first, wv});
                        }
                        if (!bw.empty()) {
                            it.pts.emplace_back(v, std::move(vec));
                            it.bw.push_back(std::move(bw));
                        }
                    }
                    if (!it.pts.empty()) plan[u].push_back(std::move(it));
                }
        }
    }
    return HEC_OK;
}

// Channel shards (Section 4.1, "With Channel Shards"): shard (f, v) holds rows
// v*R .. v*R+R-1 of channel f.  Each input shard is rotated cyclically by
// k*mp + l per tap; output shard (g, v) takes the rows whose source row lies
// in its own shard from its own rotation (mask m) and the rows whose source
// lies in shard v + sign(k) from that shard's rotation (the complement);
// rows outside the channel read the zero padding.
static hec_status conv_items_channel(const Layout &L, const double *w, uint32_t Co, uint32_t kh, uint32_t kw,
                                     uint32_t pad, Layout &out, std::vector<std::vector<ConvItem>> &plan)
{
    const int H = (int)L.H, W = (int)L.W, mp = (int)L.mp, R = (int)L.R(), spc = (int)L.spc(), N = (int)L.N;
    const int Ho = H + 2 * (int)pad - (int)kh + 1, Wo = W + 2 * (int)pad - (int)kw + 1;
    if (Ho < 1 || Wo < 1 || Ho > mp || Wo > mp) HEC_FAIL(HEC_ELAYOUT, "bad convolution geometry");
    if ((int)kh / 2 >= R) HEC_FAIL(HEC_ELAYOUT, "kernel taller than a channel shard");
    out = Layout();
    out.N = L.N; out.C = Co; out.H = Ho; out.W = Wo; out.mp = L.mp; out.channel = true;
    for (uint32_t g = 0; g < Co; g++)
        for (int v = 0; v < spc; v++) out.cs.push_back({(int32_t)g, v});
    const uint32_t Ci = L.C;
    plan.assign(L.cs.size(), {});
    std::vector<double> mask(N);
    for (size_t u = 0; u < L.cs.size(); u++) {
        const int f = L.cs[u].first, vin = L.cs[u].second;
        for (uint32_t kr = 0; kr < kh; kr++)
            for (uint32_t kc = 0; kc < kw; kc++) {
                const int dk = (int)kr - (int)pad, dl = (int)kc - (int)pad;
                int64_t a = ((int64_t)dk * mp + dl) % N;
                if (a < 0) a += N;
                ConvItem it;
                it.amount = (int32_t)a;
                it.baby = 0;
                it.giant = (int32_t)a;
                int cands[2] = {vin, dk > 0 ? vin - 1 : vin + 1};
                const int ncand = dk != 0 ? 2 : 1;
                for (int ci = 0; ci < ncand; ci++) {
                    const int v = cands[ci];
                    if (v < 0 || v >= spc) continue;
                    bool any = false;
                    for (int il = 0; il < R; il++)
                        for (int j = 0; j < mp; j++) {
                            const int gi = v * R + il, src = gi + dk;
                            const bool same = il + dk >= 0 && il + dk < R;
                            bool ok = gi < Ho && j < Wo && src >= 0 && src < H && j + dl >= 0 && j + dl < W &&
                                      (v == vin ? same : !same);
                            mask[(size_t)il * mp + j] = ok ? 1.0 : 0.0;
                            any |= ok;
                        }
                    if (!any) continue;
                    for (uint32_t g = 0; g < Co; g++) {
                        const double wv = w[(((size_t)g * Ci + f) * kh + kr) * kw + kc];
                        if (wv == 0.0) continue;
                        std::vector<double> vec(N);
                        for (int e = 0; e < N; e++) vec[e] = wv * mask[e];
                        it.pts.emplace_back(g * spc + v, std::move(vec));
                    }
                }
                if (!it.pts.empty()) plan[u].push_back(std::move(it));
            }
    }
    return HEC_OK;
}

// ---------------------------------------------------------------------------
// pooling masks (Section 4.2)
// ---------------------------------------------------------------------------
static std::vector<char> valid_blocks(const Layout &L)
{
    std::vector<char> v(L.nb(), 0);
    for (auto &m : L.maps)
        for (uint32_t b = 0; b < L.nb(); b++) v[b] |= m[b] >= 0;
    return v;
}

static std::vector<double> per_block(const Layout &L, const std::vector<double> &blk)
{
    std::vector<double> v(L.N, 0.0);
    auto vb = valid_blocks(L);
    for (uint32_t b = 0; b < L.nb(); b++)
        if (vb[b]) std::copy(blk.begin(), blk.end(), v.begin() + (size_t)b * L.B());
    return v;
}

// the three mask kinds: 'h' (rot_i of column 2i of even rows), 'v' (rot_{3j mp/2} of the
// left half of row 2j), 'f' (fused: element (2j, 2i) after rot_i)
static std::vector<double> pool_mask(const Layout &L, char kind, uint32_t i, uint32_t j, uint32_t Wo, double val,
                                     int part)
{
    if (L.channel) {
        // one shard of a channel: rows v*R + r of the channel, r < R
        const uint32_t R = L.R();
        std::vector<double> v(L.N, 0.0);
        if (kind == 'h') {
            for (uint32_t r = 0; r < R; r += 2)
                if (part * R + r < L.H) v[(size_t)r * L.mp + i] = val;
        } else if (kind == 'v') {
            uint32_t o = j * L.mp / 2;
            for (uint32_t c = 0; c < Wo; c++) v[o + c] = 1.0;
        } else if (kind == 'f') {
            v[(size_t)(2 * j) * L.mp + i] = val;
        }  // 'z': all zero
        return v;
    }
    std::vector<double> blk(L.B(), 0.0);
    if (kind == 'h') {
        for (uint32_t r = 0; r < L.H; r += 2) blk[(size_t)r * L.mp + i] = val;
    } else if (kind == 'v') {
        uint32_t o = j * L.mp / 2;
        for (uint32_t c = 0; c < Wo; c++) blk[o + c] = 1.0;
    } else {
        blk[(size_t)(2 * j) * L.mp + i] = val;
    }
    return per_block(L, blk);
}

static std::string layout_key(const Layout &L, int part)
{
    std::ostringstream s;
    s << L.N << ":" << L.C << ":" << L.H << ":" << L.W << ":" << L.mp;
    if (L.channel) {
        s << ":ch" << part;
        return s.str();
    }
    auto vb = valid_blocks(L);
    s << ":";
    for (char c : vb) s << (int)c;
    return s.str();
}

// one rotation of a ciphertext and the plaintexts its result is multiplied by,
// per output (index, plaintext)
struct RotTerm {
    int32_t amount = 0;
    std::vector<std::pair<uint32_t, hec_pt *>> pts;
    int32_t tap = -1;  // basis-mask plans: the tap whose basis polynomials the weight rows of pts combine
};

// cached mask plaintexts (they only depend on the layout, shard part, index, level and scale)
static hec_status get_masks(hec_ctx *c, const Layout &L, char kind, const std::vector<std::pair<uint32_t, uint32_t>> &ij,
                            uint32_t Wo, double val, uint32_t level, double scale, std::vector<hec_pt *> &out,
                            int part = -1, const std::vector<int32_t> *rolls = nullptr)
{
    std::string base = layout_key(L, part);
    std::vector<std::string> keys;
    std::vector<size_t> miss;
    out.assign(ij.size(), nullptr);
    for (size_t t = 0; t < ij.size(); t++) {
        std::ostringstream s;
        s << base << "|" << kind << "|" << ij[t].first << "|" << ij[t].second << "|" << Wo << "|" << val << "|"
          << level << "|" << scale << "|" << (rolls ? (*rolls)[t] : 0);
        keys.push_back(s.str());
        auto it = c->mask_cache.find(keys.back());
        if (it != c->mask_cache.end()) out[t] = it->second;
        else miss.push_back(t);
    }
    if (miss.empty()) return HEC_OK;
    std::vector<std::vector<double>> vecs;
    std::vector<const double *> zp;
    for (size_t t : miss) {
        std::vector<double> v = pool_mask(L, kind, ij[t].first, ij[t].second, Wo, val, part);
        const size_t N = v.size(), r = rolls ? (size_t)(((*rolls)[t] % (int64_t)N + N) % N) : 0;
        if (r) {
            // the mask rotated back by a giant step: slot i takes slot i - r
            std::vector<double> w(N);
            for (size_t i = 0; i < N; i++) w[(i + r) % N] = v[i];
            v.swap(w);
        }
        vecs.push_back(std::move(v));
    }
    for (auto &v : vecs) zp.push_back(v.data());
    std::vector<hec_pt *> pts;
    PoolScope ps(c, &c->pool);  // cached for the context's lifetime
    HEC_CHECK(pt_encode_many(c, zp, L.N, level, scale, pts, true));
    for (size_t a = 0; a < miss.size(); a++) {
        c->mask_cache[keys[miss[a]]] = pts[a];
        out[miss[a]] = pts[a];
    }
    return HEC_OK;
}

// ---------------------------------------------------------------------------
// small helpers over ciphertext lists
// ---------------------------------------------------------------------------
static void free_all(std::vector<hec_ct *> &v)
{
    for (auto *x : v) ct_free(x);
    v.clear();
}

static hec_status sum_into(hec_ctx *c, hec_ct *&acc, hec_ct *t)
{
    if (!acc) { acc = t; return HEC_OK; }
    hec_status s = ct_add_inplace(c, acc, t);
    ct_free(t);
    return s;
}

static hec_status rotate_list(hec_ctx *c, const hec_ct *ct, const std::vector<int32_t> &steps,
                              std::vector<hec_ct *> &out)
{
    out.assign(steps.size(), nullptr);
    if (steps.empty()) return HEC_OK;
    return ckks_rotate_hoisted(c, ct, steps.data(), steps.size(), out.data());
}

static hec_status mac_rotations(hec_ctx *c, const std::vector<hec_ct *> &rots, const std::vector<RotTerm> &its,
                                size_t i0, std::vector<hec_ct *> &acc, std::vector<char> &first, const BasisArg *bt);

// Lazy ModDown: the key-switch products of every rotation are multiplied by
// their plaintexts and summed over Q_l and P; each output then takes one
// ModDown (instead of one per rotation).  Rotations by zero enter as P * pt * ct.
// out[v] (allocated here, at the inputs' level, not rescaled) = sum over input
// u and its terms of pt * rot(in[u], amount).  Plaintexts carry the limbs of
// the special primes.
// bt (nullable): the plaintexts are weight rows of a basis-mask plan (E, nb, nqp set; taps from the terms)
static hec_status lazy_rotate_mac(hec_ctx *c, const std::vector<const hec_ct *> &in,
                                  const std::vector<std::vector<RotTerm>> &terms_of, size_t nout,
                                  std::vector<hec_ct *> &out, const BasisArg *bt = nullptr)
{
    out.assign(nout, nullptr);
    if (in.empty() || in.size() != terms_of.size()) HEC_FAIL(HEC_EINVAL, "lazy sum: inputs and terms differ");
    const size_t n = c->n;
    const uint32_t lvl = in[0]->level, nq = lvl + 1, nqp = nq + c->k;
    const uint32_t beta = (nq + c->alpha - 1) / c->alpha;
    for (auto *ct : in)
        if (ct->level != lvl) HEC_FAIL(HEC_ELEVEL, "lazy sum over inputs at different levels");
    // inputs with a rotation by a nonzero amount: their ModUps in one batch
    std::vector<const hec_ct *> mu;
    std::vector<size_t> mu_of(in.size(), SIZE_MAX);
    for (size_t u = 0; u < in.size(); u++) {
        bool rot = false;
        for (auto &it : terms_of[u]) {
            const uint32_t g = c->galois(it.amount);
            if (g != 1 && !c->rotkeys.count(g)) HEC_FAIL(HEC_ENOKEY, "no rotation key for step %d", it.amount);
            rot |= g != 1;
        }
        if (rot) {
            mu_of[u] = mu.size();
            mu.push_back(in[u]);
        }
    }
    // accumulators of all outputs in one buffer, so that their ModDowns batch
    u64 *Eall = c->alloc(nout * 2 * (size_t)nqp * n);
    if (!Eall) HEC_FAIL(HEC_ENOMEM, "accumulator allocation");
    u64 *Dall = nullptr;
    hec_status s = ct_modup_many(c, mu, &Dall);
    std::vector<char> used(nout, 0), fresh(nout, 1);
    double scale = 1.0;
    for (size_t u = 0; u < in.size() && s == HEC_OK; u++) {
        const auto &its = terms_of[u];
        if (its.empty()) continue;
        const hec_ct *ct = in[u];
        const u64 *D = mu_of[u] == SIZE_MAX ? nullptr : Dall + mu_of[u] * beta * (size_t)nqp * n;
        for (size_t v0 = 0; v0 < nout && s == HEC_OK; v0 += HEC_MAC_OUT) {
            const size_t nv = std::min((size_t)HEC_MAC_OUT, nout - v0);
            // the terms of this input with a product for an output of the group
            std::vector<size_t> terms;
            for (size_t t = 0; t < its.size(); t++)
                for (auto &pp : its[t].pts)
                    if (pp.first >= v0 && pp.first < v0 + nv) {
                        terms.push_back(t);
                        break;
                    }
            // rotations by zero first (the kernel takes them as a leading run)
            std::stable_partition(terms.begin(), terms.end(),
                                  [&](size_t t) { return c->galois(its[t].amount) == 1; });
            for (size_t b0 = 0; b0 < terms.size() && s == HEC_OK; b0 += HEC_KS_BATCH) {
                const size_t nt = std::min((size_t)HEC_KS_BATCH, terms.size() - b0);
                KsMacBatch b{};
                BasisArg ba = bt ? *bt : BasisArg{};
                int first = 0;
                for (size_t j = 0; j < nv; j++) {
                    b.E[j] = Eall + (v0 + j) * 2 * (size_t)nqp * n;
                    if (fresh[v0 + j]) first |= 1 << j;
                    fresh[v0 + j] = 0;
                }
                for (size_t t = 0; t < nt && s == HEC_OK; t++) {
                    const auto &it = its[terms[b0 + t]];
                    const uint32_t g = c->galois(it.amount);
                    b.g[t] = g;
                    b.key[t] = g == 1 ? nullptr : c->rotkeys[g];
                    b.D[t] = D;
                    b.ct[t] = ct->d;
                    if (bt) {
                        if (it.tap < 0) {
                            s = HEC_EINVAL;
                            hec_set_error("basis-mask term without a tap");
                            break;
                        }
                        ba.tap[t] = (u32)it.tap;
                    }
                    for (auto &pp : it.pts) {
                        if (pp.first < v0 || pp.first >= v0 + nv) continue;
                        if (!pp.second->has_p || pp.second->level != lvl) {
                            s = HEC_EINVAL;
                            hec_set_error("plaintexts of a lazy sum need the special-prime limbs at the level");
                            break;
                        }
                        b.pt[t][pp.first - v0] = pp.second->d;
                        used[pp.first] = 1;
                        scale = ct->scale * pp.second->scale;
                    }
                }
                if (s != HEC_OK) break;
                if (!hec_ks_mac(c->T, b, (int)nt, (int)nv, (int)beta, (int)nq, (int)nqp, c->qpmap(lvl),
                                c->d_pmodq_m, (int)c->NLK, first, c->st, bt ? &ba : nullptr)) {
                    s = HEC_EINVAL;
                    hec_set_error("invalid key-switch batch");
                }
                for (size_t t = 0; t < nt; t++) c->ks_count += b.g[t] != 1;
            }
        }
    }
    for (size_t v = 0; v < nout && s == HEC_OK; v++) {
        if (!used[v]) {
            s = HEC_ELAYOUT;
            hec_set_error("output shard %zu received no product", v);
            break;
        }
        if (!(out[v] = ct_new(c, lvl, scale))) {
            s = HEC_ENOMEM;
            hec_set_error("ciphertext allocation");
        }
    }
    if (s == HEC_OK) s = ct_moddown_many(c, lvl, Eall, out);
    c->release(Dall);
    c->release(Eall);
    if (s == HEC_OK && hipGetLastError() != hipSuccess) s = HEC_EDEVICE, hec_set_error("lazy accumulation launch");
    if (s != HEC_OK) free_all(out);
    return s;
}

// out[o] (not rescaled) = sum_t masks[o][t] * rot(ct, steps[t]): hoisted
// rotations then plaintext products, or (lazy) the same products taken on the
// key-switch outputs with one ModDown per output
static hec_status rot_masked_sums(hec_ctx *c, const hec_ct *ct, const std::vector<int32_t> &steps,
                                  const std::vector<std::vector<hec_pt *>> &masks, bool lazy,
                                  std::vector<hec_ct *> &out)
{
    out.clear();
    if (lazy) {
        std::vector<std::vector<RotTerm>> terms(1);
        for (size_t t = 0; t < steps.size(); t++) {
            RotTerm rt;
            rt.amount = steps[t];
            for (size_t o = 0; o < masks.size(); o++) rt.pts.push_back({(uint32_t)o, masks[o][t]});
            terms[0].push_back(std::move(rt));
        }
        return lazy_rotate_mac(c, {ct}, terms, masks.size(), out);
    }
    if (steps.empty()) HEC_FAIL(HEC_ELAYOUT, "masked sum without a term");
    std::vector<hec_ct *> rots;
    HEC_CHECK(rotate_list(c, ct, steps, rots));
    // every output's products and sums as plaintext-product batches (exact
    // sums, one reduction per output: the residues of one MAC at a time)
    const size_t no = masks.size();
    hec_status s = HEC_OK;
    out.assign(no, nullptr);
    for (size_t o = 0; o < no && s == HEC_OK; o++)
        if (!(out[o] = ct_new(c, rots[0]->level, 1.0))) s = HEC_ENOMEM, hec_set_error("ciphertext allocation");
    std::vector<RotTerm> its(rots.size());
    for (size_t t = 0; t < rots.size(); t++) {
        its[t].amount = steps[t];
        for (size_t o = 0; o < no; o++) its[t].pts.push_back({(uint32_t)o, masks[o][t]});
    }
    std::vector<char> first(no, 1);
    if (s == HEC_OK) s = mac_rotations(c, rots, its, 0, out, first, nullptr);
    free_all(rots);
    if (s != HEC_OK) free_all(out);
    return s;
}

// ---------------------------------------------------------------------------
// downsample / consolidate / duplicate
// ---------------------------------------------------------------------------
// out (allocated here, not rescaled) = sum over terms of rot(ct_t, amount_t)
// for ciphertexts at one level and scale, with lazy ModDown: every rotated
// ciphertext takes its own ModUp, the key-switch products are summed over Q_l
// and P, and the sum takes one ModDown.
typedef std::vector<std::pair<const hec_ct *, int32_t>> RotSum;
static hec_status lazy_rotation_sums(hec_ctx *c, const std::vector<RotSum> &sums, std::vector<hec_ct *> &out)
{
    const size_t nout = sums.size();
    out.assign(nout, nullptr);
    if (!nout) return HEC_OK;
    for (auto &sm : sums)
        if (sm.empty()) HEC_FAIL(HEC_EINVAL, "empty rotation sum");
    const size_t n = c->n;
    const uint32_t lvl = sums[0][0].first->level, nq = lvl + 1, nqp = nq + c->k;
    const uint32_t beta = (nq + c->alpha - 1) / c->alpha;
    // the distinct ciphertexts rotated by a nonzero amount: their ModUps in one batch
    std::vector<const hec_ct *> mu;
    std::map<const hec_ct *, size_t> mi;
    for (auto &sm : sums) {
        const double scale = sm[0].first->scale;
        for (auto &t : sm) {
            if (t.first->level != lvl || t.first->scale != scale)
                HEC_FAIL(HEC_ELEVEL, "rotation sum over different levels or scales");
            const uint32_t g = c->galois(t.second);
            if (g == 1) continue;
            if (!c->rotkeys.count(g)) HEC_FAIL(HEC_ENOKEY, "no rotation key for step %d", t.second);
            if (!mi.count(t.first)) {
                mi[t.first] = mu.size();
                mu.push_back(t.first);
            }
        }
    }
    const u64 *one = ones_qp(c, lvl);
    u64 *Eall = c->alloc(nout * 2 * (size_t)nqp * n);
    if (!one || !Eall) {
        c->release(Eall);
        HEC_FAIL(HEC_ENOMEM, "rotation-sum buffers");
    }
    u64 *Dall = nullptr;
    hec_status s = ct_modup_many(c, mu, &Dall);
    for (size_t v = 0; v < nout && s == HEC_OK; v++) {
        RotSum terms = sums[v];
        std::stable_partition(terms.begin(), terms.end(),
                              [&](const std::pair<const hec_ct *, int32_t> &t) { return c->galois(t.second) == 1; });
        for (size_t b0 = 0; b0 < terms.size() && s == HEC_OK; b0 += HEC_KS_BATCH) {
            const size_t nt = std::min((size_t)HEC_KS_BATCH, terms.size() - b0);
            KsMacBatch b{};
            b.E[0] = Eall + v * 2 * (size_t)nqp * n;
            for (size_t t = 0; t < nt; t++) {
                const hec_ct *ct = terms[b0 + t].first;
                const uint32_t g = c->galois(terms[b0 + t].second);
                b.g[t] = g;
                b.ct[t] = ct->d;
                b.pt[t][0] = one;
                if (g != 1) {
                    b.D[t] = Dall + mi[ct] * beta * (size_t)nqp * n;
                    b.key[t] = c->rotkeys[g];
                    c->ks_count++;
                }
            }
            if (!hec_ks_mac(c->T, b, (int)nt, 1, (int)beta, (int)nq, (int)nqp, c->qpmap(lvl), c->d_pmodq_m,
                            (int)c->NLK, b0 == 0 ? 1 : 0, c->st)) {
                s = HEC_EINVAL;
                hec_set_error("invalid key-switch batch");
            }
        }
    }
    for (size_t v = 0; v < nout && s == HEC_OK; v++)
        if (!(out[v] = ct_new(c, lvl, sums[v][0].first->scale))) s = HEC_ENOMEM, hec_set_error("ciphertext allocation");
    if (s == HEC_OK) s = ct_moddown_many(c, lvl, Eall, out);
    c->release(Dall);
    c->release(Eall);
    if (s != HEC_OK) free_all(out);
    return s;
}

// Baby / giant split of rotation amounts steps[t] = idx_t * unit: with
// G = ceil(sqrt(max idx + 1)), baby = (idx mod G) * unit, giant = (idx - idx mod G) * unit.
static void bsgs_split(const std::vector<int32_t> &steps, int32_t unit, std::vector<int32_t> &baby,
                       std::vector<int32_t> &giant)
{
    int32_t n = 1;
    for (int32_t a : steps) n = std::max(n, a / unit + 1);
    int32_t G = 1;
    while (G * G < n) G++;
    baby.clear();
    giant.clear();
    for (int32_t a : steps) {
        const int32_t i = a / unit;
        baby.push_back((i % G) * unit);
        giant.push_back((i - i % G) * unit);
    }
}

// Baby-step / giant-step evaluation (double hoisting): T_k = lazy sums of the
// baby terms of every input (one ModDown per k), then output v = the lazy sum
// of rot_{gv[k].first}(T_k) over the k with gv[k].second == v.  Not rescaled.
static hec_status bsgs_eval(hec_ctx *c, const std::vector<const hec_ct *> &ins,
                            const std::vector<std::vector<RotTerm>> &babies,
                            const std::vector<std::pair<int32_t, uint32_t>> &gv, size_t nout,
                            std::vector<hec_ct *> &out)
{
    out.assign(nout, nullptr);
    std::vector<hec_ct *> T;
    HEC_CHECK(lazy_rotate_mac(c, ins, babies, gv.size(), T));
    std::vector<RotSum> sums(nout);
    for (size_t k = 0; k < gv.size(); k++)
        if (gv[k].second < nout) sums[gv[k].second].push_back({T[k], gv[k].first});
    hec_status s = HEC_OK;
    for (size_t v = 0; v < nout && s == HEC_OK; v++)
        if (sums[v].empty()) s = HEC_ELAYOUT, hec_set_error("output %zu received no product", v);
    if (s == HEC_OK) s = lazy_rotation_sums(c, sums, out);
    free_all(T);
    if (s != HEC_OK) free_all(out);
    return s;
}

// out[o] (not rescaled) = sum_t masks[o][t] * rot(ct, baby[t] + giant[t]) by
// baby and giant steps; masks[o][t] must already be rotated back by giant[t]
static hec_status bsgs_masked_sums(hec_ctx *c, const hec_ct *ct, const std::vector<int32_t> &baby,
                                   const std::vector<int32_t> &giant,
                                   const std::vector<std::vector<hec_pt *>> &masks, std::vector<hec_ct *> &out)
{
    std::map<std::pair<int32_t, uint32_t>, uint32_t> idx;
    for (size_t t = 0; t < baby.size(); t++)
        for (size_t o = 0; o < masks.size(); o++) idx[{giant[t], (uint32_t)o}] = 0;
    std::vector<std::pair<int32_t, uint32_t>> gv;
    for (auto &kv : idx) {
        kv.second = (uint32_t)gv.size();
        gv.push_back(kv.first);
    }
    std::map<int32_t, RotTerm> byb;
    for (size_t t = 0; t < baby.size(); t++) {
        RotTerm &rt = byb[baby[t]];
        rt.amount = baby[t];
        for (size_t o = 0; o < masks.size(); o++) rt.pts.push_back({idx[{giant[t], (uint32_t)o}], masks[o][t]});
    }
    std::vector<std::vector<RotTerm>> babies(1);
    for (auto &kv : byb) babies[0].push_back(kv.second);
    return bsgs_eval(c, {ct}, babies, gv, masks.size(), out);
}

// One masked-sum stage of the pooling in evaluation mode `mode` (0 per
// rotation, 2 lazy ModDown, 3 baby-step / giant-step); masks[o][t] are fetched
// by get_mask(o, rolls) with the giant-step rolls in mode 3 (null otherwise).
// Sums of fewer than BSGS_MIN_STEPS rotations stay lazy in mode 3: below that
// the ModUp/ModDown of the giant sums cost more than the key switches saved.
#define BSGS_MIN_STEPS 32
template <class GetMasks>
static hec_status pool_stage(hec_ctx *c, const hec_ct *ct, const std::vector<int32_t> &steps, int32_t unit,
                             size_t nout, int mode, GetMasks get_masks_for, std::vector<hec_ct *> &out)
{
    std::vector<std::vector<hec_pt *>> masks(nout);
    if (mode == 3 && steps.size() < BSGS_MIN_STEPS) mode = 2;
    if (mode == 3) {
        std::vector<int32_t> baby, giant;
        bsgs_split(steps, unit, baby, giant);
        for (size_t o = 0; o < nout; o++) HEC_CHECK(get_masks_for(o, &giant, masks[o]));
        return bsgs_masked_sums(c, ct, baby, giant, masks, out);
    }
    for (size_t o = 0; o < nout; o++) HEC_CHECK(get_masks_for(o, nullptr, masks[o]));
    return rot_masked_sums(c, ct, steps, masks, mode == 2, out);
}

// Reduction of one shard after its 2x2 sums D (Section 4.2): column 2i of the
// kept rows to column i (hs = 0..Wo-1), then row 2j to row j (js, shifts
// 3j*mp/2), each a masked sum of hoisted rotations and a rescale; fused (one
// level left) takes both in one masked sum per row at scale q/4.  `part` >= 0
// selects the masks of a channel shard.
static hec_status pool_reduce(hec_ctx *c, const hec_ct *D, const Layout &L, const std::vector<int32_t> &hs,
                              const std::vector<uint32_t> &js, uint32_t Wo, double val, uint32_t lvl, bool fused,
                              int mode, int part, hec_ct **out)
{
    *out = nullptr;
    const uint32_t mp = L.mp;
    if (fused) {
        std::vector<hec_ct *> T;
        HEC_CHECK(pool_stage(c, D, hs, 1, js.size(), mode,
                             [&](size_t t, const std::vector<int32_t> *rolls, std::vector<hec_pt *> &m) {
                                 std::vector<std::pair<uint32_t, uint32_t>> ij;
                                 for (uint32_t i = 0; i < Wo; i++) ij.push_back({i, js[t]});
                                 return get_masks(c, L, 'f', ij, Wo, val, lvl, (double)c->mod[lvl] / 4.0, m, part,
                                                  rolls);
                             },
                             T));
        hec_ct *acc = nullptr;
        hec_status s = HEC_OK;
        for (size_t t = 0; t < js.size(); t++) {
            hec_ct *x = T[t];
            T[t] = nullptr;
            if (s == HEC_OK && js[t] > 0) {
                hec_ct *m = nullptr;
                s = ckks_rotate(c, x, (int32_t)(3 * js[t] * mp / 2), &m);
                ct_free(x);
                x = m;
            }
            if (s == HEC_OK) s = sum_into(c, acc, x);
            else ct_free(x);
        }
        if (s == HEC_OK) s = ct_rescale(c, acc);
        if (s != HEC_OK) { ct_free(acc); return s; }
        *out = acc;
        return HEC_OK;
    }
    std::vector<std::pair<uint32_t, uint32_t>> ij, jj;
    for (uint32_t i = 0; i < Wo; i++) ij.push_back({i, 0});
    std::vector<hec_ct *> M1;
    HEC_CHECK(pool_stage(c, D, hs, 1, 1, mode,
                         [&](size_t, const std::vector<int32_t> *rolls, std::vector<hec_pt *> &m) {
                             return get_masks(c, L, 'h', ij, Wo, val, lvl, (double)c->mod[lvl], m, part, rolls);
                         },
                         M1));
    hec_status s = ct_rescale(c, M1[0]);
    if (s == HEC_OK && M1[0]->level < 1) s = HEC_ELEVEL, hec_set_error("separable pooling needs two levels");
    if (s != HEC_OK) { free_all(M1); return s; }
    const uint32_t l1 = M1[0]->level;
    std::vector<int32_t> vs;
    for (uint32_t j : js) {
        vs.push_back((int32_t)(3 * j * mp / 2));
        jj.push_back({0, j});
    }
    std::vector<hec_ct *> M2;
    s = pool_stage(c, M1[0], vs, (int32_t)(3 * mp / 2), 1, mode,
                   [&](size_t, const std::vector<int32_t> *rolls, std::vector<hec_pt *> &m) {
                       return get_masks(c, L, 'v', jj, Wo, 1.0, l1, (double)c->mod[l1], m, part, rolls);
                   },
                   M2);
    free_all(M1);
    HEC_CHECK(s);
    s = ct_rescale(c, M2[0]);
    if (s != HEC_OK) { free_all(M2); return s; }
    *out = M2[0];
    return HEC_OK;
}

static hec_status downsample(hec_ctx *c, const std::vector<hec_ct *> &in, const Layout &L, bool select,
                             int mode, std::vector<hec_ct *> &out, Layout &nl)
{
    const uint32_t mp = L.mp;
    uint32_t Ho, Wo;
    double val;
    if (select) {
        Ho = (L.H + 1) / 2; Wo = (L.W + 1) / 2; val = 1.0;
    } else {
        if (L.H % 2 || L.W % 2) HEC_FAIL(HEC_ELAYOUT, "average pooling needs even H and W");
        Ho = L.H / 2; Wo = L.W / 2; val = 0.25;
    }
    out.clear();
    for (hec_ct *ct : in) {
        const uint32_t lvl = ct->level;
        if (lvl < 1) HEC_FAIL(HEC_ELEVEL, "pooling needs a level");
        const bool fused = lvl < 2;
        hec_ct *D = nullptr;
        if (!select) {
            std::vector<hec_ct *> r;
            HEC_CHECK(rotate_list(c, ct, {1, (int32_t)mp, (int32_t)mp + 1}, r));
            D = ct_clone(c, ct);
            for (auto *x : r) HEC_CHECK(sum_into(c, D, x));
        } else {
            D = ct_clone(c, ct);
        }
        std::vector<int32_t> hs;
        for (uint32_t i = 0; i < Wo; i++) hs.push_back((int32_t)i);
        std::vector<uint32_t> js;
        for (uint32_t j = 0; j < Ho; j++) js.push_back(j);
        hec_ct *o = nullptr;
        hec_status s = pool_reduce(c, D, L, hs, js, Wo, val, lvl, fused, mode, -1, &o);
        ct_free(D);
        HEC_CHECK(s);
        out.push_back(o);
    }
    nl = Layout();
    nl.N = L.N; nl.C = L.C; nl.H = Ho; nl.W = Wo; nl.mp = mp / 2;
    for (auto &m : L.maps) {
        std::vector<int32_t> nm(4 * L.nb(), -1);
        for (uint32_t b = 0; b < L.nb(); b++) nm[4 * b] = m[b];
        nl.maps.push_back(nm);
    }
    return HEC_OK;
}

static hec_status duplicate(hec_ctx *c, hec_ct *ct, Layout &L, uint32_t d, hec_ct **out)
{
    const int32_t Bn = (int32_t)L.B();
    const uint32_t step = 4 / d;
    std::vector<int32_t> sh;
    for (uint32_t m = 1; m < d; m++) sh.push_back(-(int32_t)(m * step) * Bn);
    std::vector<hec_ct *> r;
    HEC_CHECK(rotate_list(c, ct, sh, r));
    hec_ct *acc = ct_clone(c, ct);
    for (auto *x : r) HEC_CHECK(sum_into(c, acc, x));
    std::vector<int32_t> lam = L.maps[0];
    for (uint32_t b = 0; b < L.nb() / 4; b++)
        for (uint32_t m = 1; m < d; m++)
            for (uint32_t e = 0; e < step; e++) lam[4 * b + m * step + e] = lam[4 * b + e];
    L.maps[0] = lam;
    *out = acc;
    return HEC_OK;
}

// Channel shards are downsampled one by one (Section 4.2, "With Channel
// Shards"): 2x2 sums stay inside a shard (R is even), column 2i of the even
// rows that belong to the channel goes to column i, the left half of local row
// 2j to j*mp/2.  A shard below the channel's last row pools to zero.
static hec_status downsample_channel(hec_ctx *c, const std::vector<hec_ct *> &in, const Layout &L, bool select,
                                     int mode, std::vector<hec_ct *> &out)
{
    const uint32_t mp = L.mp, R = L.R();
    uint32_t Wo;
    double val;
    if (select) {
        Wo = (L.W + 1) / 2; val = 1.0;
    } else {
        if (L.H % 2 || L.W % 2) HEC_FAIL(HEC_ELAYOUT, "average pooling needs even H and W");
        Wo = L.W / 2; val = 0.25;
    }
    out.clear();
    for (size_t u = 0; u < in.size(); u++) {
        hec_ct *ct = in[u];
        const int part = L.cs[u].second;
        const uint32_t lvl = ct->level;
        if (lvl < 1) HEC_FAIL(HEC_ELEVEL, "pooling needs a level");
        const bool fused = lvl < 2;
        std::vector<uint32_t> js;
        for (uint32_t r = 0; r < R; r += 2)
            if (part * R + r < L.H) js.push_back(r / 2);
        std::vector<hec_pt *> pts;
        if (js.empty()) {
            HEC_CHECK(get_masks(c, L, 'z', {{0, 0}}, Wo, val, lvl, fused ? (double)c->mod[lvl] / 4.0 : (double)c->mod[lvl],
                                pts, part));
            hec_ct *a = ct_new(c, lvl, 1.0);
            if (!a) HEC_FAIL(HEC_ENOMEM, "ciphertext allocation");
            HEC_CHECK(ct_mac_pt(c, a, ct, pts[0], true));
            HEC_CHECK(ct_rescale(c, a));
            if (!fused) {
                HEC_CHECK(get_masks(c, L, 'z', {{0, 0}}, Wo, val, a->level, (double)c->mod[a->level], pts, part));
                hec_ct *b = ct_new(c, a->level, 1.0);
                if (!b) HEC_FAIL(HEC_ENOMEM, "ciphertext allocation");
                HEC_CHECK(ct_mac_pt(c, b, a, pts[0], true));
                ct_free(a);
                HEC_CHECK(ct_rescale(c, b));
                a = b;
            }
            out.push_back(a);
            continue;
        }
        hec_ct *D = ct_clone(c, ct);
        if (!select) {
            std::vector<hec_ct *> r;
            HEC_CHECK(rotate_list(c, ct, {1, (int32_t)mp, (int32_t)mp + 1}, r));
            for (auto *x : r) HEC_CHECK(sum_into(c, D, x));
        }
        std::vector<int32_t> hs;
        for (uint32_t i = 0; i < Wo; i++) hs.push_back((int32_t)i);
        hec_ct *o = nullptr;
        hec_status s = pool_reduce(c, D, L, hs, js, Wo, val, lvl, fused, mode, part, &o);
        ct_free(D);
        HEC_CHECK(s);
        out.push_back(o);
    }
    return HEC_OK;
}

// Consolidate every four consecutive downsampled channel shards (shifts by
// multiples of N/4).  The result is channel-sharded again while a pooled
// channel still exceeds N slots, image-sharded otherwise; one channel in two
// shards is duplicated by two.  No permutation arises.
static hec_status merge_channel(hec_ctx *c, std::vector<hec_ct *> &ds, const Layout &L, uint32_t H2, uint32_t W2,
                                std::vector<hec_ct *> &out, Layout &ol)
{
    const uint32_t N = L.N, q4 = N / 4;
    const size_t t = ds.size();
    out.clear();
    std::vector<std::vector<std::pair<int32_t, int32_t>>> groups;
    for (size_t s0 = 0; s0 < t; s0 += 4) {
        const size_t g = std::min((size_t)4, t - s0);
        hec_ct *acc = ct_clone(c, ds[s0]);
        for (size_t e = 1; e < g; e++) {
            hec_ct *r = nullptr;
            HEC_CHECK(ckks_rotate(c, ds[s0 + e], -(int32_t)(e * q4), &r));
            HEC_CHECK(sum_into(c, acc, r));
        }
        groups.push_back(std::vector<std::pair<int32_t, int32_t>>(L.cs.begin() + s0, L.cs.begin() + s0 + g));
        out.push_back(acc);
    }
    ol = Layout();
    ol.N = N; ol.C = L.C; ol.H = H2; ol.W = W2; ol.mp = L.mp / 2;
    const uint32_t B2 = ol.B();
    if (B2 > N) {
        ol.channel = true;
        for (auto &grp : groups) ol.cs.push_back({grp[0].first, grp[0].second / 4});
        return HEC_OK;
    }
    const uint32_t nb = N / B2, per_ch = B2 / q4;
    for (auto &grp : groups) {
        std::vector<int32_t> lam(nb, -1);
        for (size_t e = 0; e < grp.size(); e++) lam[e / per_ch] = grp[e].first;
        ol.maps.push_back(lam);
    }
    if (t == 2) {  // one channel in two shards: duplicate x2
        hec_ct *r = nullptr;
        HEC_CHECK(ckks_rotate(c, out[0], -(int32_t)(N / 2), &r));
        HEC_CHECK(sum_into(c, out[0], r));
        ol.maps[0] = std::vector<int32_t>(nb, ol.maps[0][0]);
    }
    return HEC_OK;
}

// out[u] = sum_t masks[t] * rot(ins[u], steps[t]) for every input u at once:
// the nonzero rotations of all inputs amount by amount (ct_rotate_multi), the
// products and sums as plaintext-product batches (mac_rotations).  The same
// rotations and the same exact sums as one masked sum per input (mode 0).
static hec_status masked_sums_multi(hec_ctx *c, const std::vector<const hec_ct *> &ins,
                                    const std::vector<int32_t> &steps, const std::vector<hec_pt *> &masks,
                                    std::vector<hec_ct *> &out)
{
    const size_t S = ins.size();
    out.assign(S, nullptr);
    for (size_t u = 0; u < S; u++)
        if (!(out[u] = ct_new(c, ins[u]->level, 1.0))) {
            free_all(out);
            HEC_FAIL(HEC_ENOMEM, "ciphertext allocation");
        }
    std::vector<char> first(S, 1);
    std::vector<hec_ct *> zr;
    std::vector<RotTerm> zi;
    std::vector<int32_t> amounts;
    std::vector<size_t> tidx;
    for (size_t t = 0; t < steps.size(); t++) {
        if (c->galois(steps[t]) != 1) {
            amounts.push_back(steps[t]);
            tidx.push_back(t);
            continue;
        }
        for (size_t u = 0; u < S; u++) {
            zr.push_back(const_cast<hec_ct *>(ins[u]));
            RotTerm rt;
            rt.amount = steps[t];
            rt.pts.push_back({(uint32_t)u, masks[t]});
            zi.push_back(std::move(rt));
        }
    }
    hec_status s = zr.empty() ? HEC_OK : mac_rotations(c, zr, zi, 0, out, first, nullptr);
    for (size_t u0 = 0; u0 < S && s == HEC_OK && !amounts.empty(); u0 += HEC_MULTI_MAX_INPUTS) {
        const size_t G = std::min((size_t)HEC_MULTI_MAX_INPUTS, S - u0);
        std::vector<const hec_ct *> grp(ins.begin() + u0, ins.begin() + u0 + G);
        const uint64_t all = G == 64 ? ~0ull : ((1ull << G) - 1);
        std::vector<uint64_t> want(amounts.size(), all);
        auto sink = [&](size_t a0, size_t na, const std::vector<hec_ct *> &rots) -> hec_status {
            std::vector<hec_ct *> rs;
            std::vector<RotTerm> its;
            for (size_t u = 0; u < G; u++)
                for (size_t t = 0; t < na; t++) {
                    rs.push_back(rots[t * G + u]);
                    RotTerm rt;
                    rt.amount = amounts[a0 + t];
                    rt.pts.push_back({(uint32_t)(u0 + u), masks[tidx[a0 + t]]});
                    its.push_back(std::move(rt));
                }
            return mac_rotations(c, rs, its, 0, out, first, nullptr);
        };
        s = ct_rotate_multi(c, grp, amounts, want, (size_t)hec_tune_params().ks_amounts, sink);
    }
    for (size_t u = 0; u < S && s == HEC_OK; u++)
        if (first[u]) s = HEC_ELAYOUT, hec_set_error("masked sum without a term");
    if (s != HEC_OK) free_all(out);
    return s;
}

// The lazy form (reading of mode 2) of the same masked sums for every input
// at once: out[u] = ModDown(sum_t masks[t] * KS_t(ins[u])) with the key-switch
// products taken over Q_l and P and one ModDown per input (P * mask * c0 for
// rotations by zero).  The inputs are gathered into one buffer so that one
// fused key-switch launch per batch of 16 amounts covers all of them with each
// key and mask limb read once (hec_ks_mac_shards); the same sums, so the same
// ciphertexts as one lazy masked sum per input.
static hec_status masked_sums_lazy_multi(hec_ctx *c, const std::vector<const hec_ct *> &ins,
                                         const std::vector<int32_t> &steps, const std::vector<hec_pt *> &masks,
                                         std::vector<hec_ct *> &out)
{
    out.clear();
    const size_t n = c->n, S0 = ins.size();
    const uint32_t lvl = ins[0]->level, nq = lvl + 1, nqp = nq + c->k;
    const uint32_t beta = (nq + c->alpha - 1) / c->alpha;
    std::vector<size_t> order;  // rotations by zero first (the kernel takes them as a leading run)
    for (size_t t = 0; t < steps.size(); t++)
        if (c->galois(steps[t]) == 1) order.push_back(t);
    for (size_t t = 0; t < steps.size(); t++) {
        const uint32_t g = c->galois(steps[t]);
        if (g == 1) continue;
        if (!c->rotkeys.count(g)) HEC_FAIL(HEC_ENOKEY, "no rotation key for step %d", steps[t]);
        order.push_back(t);
    }
    for (auto *m : masks)
        if (!m->has_p || m->level != lvl) HEC_FAIL(HEC_EINVAL, "masks of a lazy sum need the special-prime limbs");
    const size_t G = 32;  // inputs per launch group
    hec_status s = HEC_OK;
    for (size_t u0 = 0; u0 < S0 && s == HEC_OK; u0 += G) {
        const size_t S = std::min(G, S0 - u0);
        const size_t cs = 2ull * nq * n, ds = (size_t)beta * nqp * n, es = 2ull * nqp * n;
        u64 *buf = c->alloc(S * cs), *E = c->alloc(S * es);
        if (!buf || !E) {
            c->release(buf);
            c->release(E);
            s = HEC_ENOMEM;
            hec_set_error("lazy masked sum buffers");
            break;
        }
        std::vector<hec_ct> views(S);
        std::vector<const hec_ct *> vp(S);
        for (size_t u = 0; u < S && s == HEC_OK; u++) {
            if (ins[u0 + u]->level != lvl) s = HEC_ELEVEL, hec_set_error("lazy sum over inputs at different levels");
            else if (hipMemcpyAsync(buf + u * cs, ins[u0 + u]->d, cs * 8, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
                s = HEC_EDEVICE, hec_set_error("input gather");
            views[u] = *ins[u0 + u];
            views[u].d = buf + u * cs;
            vp[u] = &views[u];
        }
        u64 *Dall = nullptr;
        if (s == HEC_OK) s = ct_modup_many(c, vp, &Dall);
        for (size_t b0 = 0; b0 < order.size() && s == HEC_OK; b0 += HEC_KS_BATCH) {
            const size_t nt = std::min((size_t)HEC_KS_BATCH, order.size() - b0);
            KsMacBatch b{};
            b.E[0] = E;
            for (size_t t = 0; t < nt; t++) {
                const size_t ti = order[b0 + t];
                const uint32_t g = c->galois(steps[ti]);
                b.g[t] = g;
                b.key[t] = g == 1 ? nullptr : c->rotkeys[g];
                b.D[t] = Dall;
                b.ct[t] = buf;
                b.pt[t][0] = masks[ti]->d;
                if (g != 1) c->ks_count += S;
            }
            if (!hec_ks_mac_shards(c->T, b, (int)nt, (int)beta, (int)nq, (int)nqp, c->qpmap(lvl), c->d_pmodq_m,
                                   (int)c->NLK, b0 == 0 ? 1 : 0, ShardArg{(u32)S, ds, cs, es}, c->st))
                s = HEC_EINVAL, hec_set_error("invalid multi-input key-switch batch");
        }
        std::vector<hec_ct *> o(S, nullptr);
        for (size_t u = 0; u < S && s == HEC_OK; u++)
            if (!(o[u] = ct_new(c, lvl, ins[u0 + u]->scale * masks[order[0]]->scale)))
                s = HEC_ENOMEM, hec_set_error("ciphertext allocation");
        if (s == HEC_OK) s = ct_moddown_many(c, lvl, E, o);
        c->release(Dall);
        c->release(buf);
        c->release(E);
        if (s == HEC_OK) out.insert(out.end(), o.begin(), o.end());
        else free_all(o);
    }
    if (s != HEC_OK) free_all(out);
    return s;
}

// Pooling mode 4 on image shards with two levels or more (Section 4.2): the
// 2x2 window sums, the horizontal and the vertical masked reductions of all
// shards together, stage by stage, each rotation key read once per stage for
// all shards; the same ciphertexts as mode 0.  Other layouts: false in *done.
static hec_status downsample_multi(hec_ctx *c, const std::vector<hec_ct *> &in, const Layout &L, bool select,
                                   std::vector<hec_ct *> &out, Layout &nl, bool *done, bool lazy = false)
{
    *done = false;
    if (L.channel || in.empty()) return HEC_OK;
    const uint32_t lvl = in[0]->level;
    for (auto *ct : in)
        if (ct->level != lvl) return HEC_OK;
    if (lvl < 2) return HEC_OK;  // the fused one-level reduction stays per shard
    const uint32_t mp = L.mp;
    uint32_t Ho, Wo;
    double val;
    if (select) {
        Ho = (L.H + 1) / 2; Wo = (L.W + 1) / 2; val = 1.0;
    } else {
        if (L.H % 2 || L.W % 2) HEC_FAIL(HEC_ELAYOUT, "average pooling needs even H and W");
        Ho = L.H / 2; Wo = L.W / 2; val = 0.25;
    }
    const size_t S = in.size();
    std::vector<hec_ct *> D(S, nullptr);
    for (size_t u = 0; u < S; u++)
        if (!(D[u] = ct_clone(c, in[u]))) { free_all(D); HEC_FAIL(HEC_ENOMEM, "ciphertext allocation"); }
    std::vector<const hec_ct *> ins(in.begin(), in.end());
    hec_status s = HEC_OK;
    if (!select) {
        // D = M + M<<1 + M<<mp + M<<(mp+1)
        const std::vector<int32_t> win = {1, (int32_t)mp, (int32_t)mp + 1};
        for (size_t u0 = 0; u0 < S && s == HEC_OK; u0 += HEC_MULTI_MAX_INPUTS) {
            const size_t G = std::min((size_t)HEC_MULTI_MAX_INPUTS, S - u0);
            std::vector<const hec_ct *> grp(ins.begin() + u0, ins.begin() + u0 + G);
            std::vector<uint64_t> want(win.size(), G == 64 ? ~0ull : ((1ull << G) - 1));
            s = ct_rotate_multi(c, grp, win, want, (size_t)hec_tune_params().ks_amounts,
                                [&](size_t, size_t na, const std::vector<hec_ct *> &rots) -> hec_status {
                                    for (size_t t = 0; t < na; t++)
                                        for (size_t u = 0; u < G; u++)
                                            HEC_CHECK(ct_add_inplace(c, D[u0 + u], rots[t * G + u]));
                                    return HEC_OK;
                                });
        }
    }
    std::vector<int32_t> hs, vs;
    std::vector<std::pair<uint32_t, uint32_t>> ij, jj;
    for (uint32_t i = 0; i < Wo; i++) {
        hs.push_back((int32_t)i);
        ij.push_back({i, 0});
    }
    for (uint32_t j = 0; j < Ho; j++) {
        vs.push_back((int32_t)(3 * j * mp / 2));
        jj.push_back({0, j});
    }
    std::vector<hec_pt *> mh, mv;
    std::vector<hec_ct *> M1, M2;
    if (s == HEC_OK) s = get_masks(c, L, 'h', ij, Wo, val, lvl, (double)c->mod[lvl], mh);
    if (s == HEC_OK) {
        const std::vector<const hec_ct *> Dc(D.begin(), D.end());
        s = lazy ? masked_sums_lazy_multi(c, Dc, hs, mh, M1) : masked_sums_multi(c, Dc, hs, mh, M1);
    }
    free_all(D);
    for (size_t u = 0; u < M1.size() && s == HEC_OK; u++) s = ct_rescale(c, M1[u]);
    const uint32_t l1 = lvl - 1;
    if (s == HEC_OK) s = get_masks(c, L, 'v', jj, Wo, 1.0, l1, (double)c->mod[l1], mv);
    if (s == HEC_OK) {
        const std::vector<const hec_ct *> Mc(M1.begin(), M1.end());
        s = lazy ? masked_sums_lazy_multi(c, Mc, vs, mv, M2) : masked_sums_multi(c, Mc, vs, mv, M2);
    }
    free_all(M1);
    for (size_t u = 0; u < M2.size() && s == HEC_OK; u++) s = ct_rescale(c, M2[u]);
    if (s != HEC_OK) {
        free_all(M2);
        return s;
    }
    out = M2;
    nl = Layout();
    nl.N = L.N; nl.C = L.C; nl.H = Ho; nl.W = Wo; nl.mp = mp / 2;
    for (auto &m : L.maps) {
        std::vector<int32_t> nm(4 * L.nb(), -1);
        for (uint32_t b = 0; b < L.nb(); b++) nm[4 * b] = m[b];
        nl.maps.push_back(nm);
    }
    *done = true;
    return HEC_OK;
}

static hec_status downsample_and_merge(hec_ctx *c, const std::vector<hec_ct *> &in, const Layout &L, bool select,
                                       int mode, std::vector<hec_ct *> &out, Layout &ol);

// Consolidation of downsampled image shards (layout nl) into groups of four
// and duplication when one or two were downsampled (Section 4.2); ds consumed.
static hec_status merge_downsampled(hec_ctx *c, std::vector<hec_ct *> &ds, const Layout &nl,
                                    std::vector<hec_ct *> &out, Layout &ol)
{
    const size_t t = ds.size();
    out.clear();
    if (t == 1) {
        hec_ct *o = nullptr;
        Layout dl = nl;
        hec_status s = duplicate(c, ds[0], dl, 4, &o);
        free_all(ds);
        HEC_CHECK(s);
        out.push_back(o);
        ol = dl;
        return HEC_OK;
    }
    const int32_t Bn = (int32_t)nl.B();
    Layout cl = nl;
    cl.maps.clear();
    for (size_t s0 = 0; s0 < t; s0 += 4) {
        const size_t g = std::min((size_t)4, t - s0);  // short last group when t % 4 != 0
        hec_ct *acc = ct_clone(c, ds[s0]);
        for (size_t e = 1; e < g; e++) {
            hec_ct *r = nullptr;
            HEC_CHECK(ckks_rotate(c, ds[s0 + e], -(int32_t)e * Bn, &r));
            HEC_CHECK(sum_into(c, acc, r));
        }
        std::vector<int32_t> lam(nl.nb(), -1);
        for (size_t e = 0; e < g; e++)
            for (uint32_t b = 0; b < nl.nb() / 4; b++) lam[4 * b + e] = nl.maps[s0 + e][4 * b];
        cl.maps.push_back(lam);
        out.push_back(acc);
    }
    free_all(ds);
    if (t == 2) {
        hec_ct *o = nullptr;
        HEC_CHECK(duplicate(c, out[0], cl, 2, &o));
        free_all(out);
        out.push_back(o);
    }
    ol = cl;
    return HEC_OK;
}

// Downsampling (and consolidation) of several images of one layout: in mode
// 4 the stages of image-sharded layouts run over the shards of all images
// together (one key read per stage for all of them), then every image is
// consolidated on its own; otherwise image by image.  Same ciphertexts as one
// downsample_and_merge per image.
static hec_status downsample_and_merge_multi(hec_ctx *c, const std::vector<std::vector<hec_ct *>> &ins,
                                             const Layout &L, bool select, int mode,
                                             std::vector<std::vector<hec_ct *>> &outs, Layout &ol)
{
    outs.assign(ins.size(), {});
    if (L.channel || (mode != 4 && mode != 2) || ins.size() == 1) {
        for (size_t r = 0; r < ins.size(); r++) {
            hec_status s = downsample_and_merge(c, ins[r], L, select, mode, outs[r], ol);
            if (s != HEC_OK) {
                for (auto &v : outs) free_all(v);
                return s;
            }
        }
        return HEC_OK;
    }
    const size_t t = ins[0].size();
    std::vector<hec_ct *> all;
    Layout Lk = L;
    Lk.maps.clear();
    for (auto &v : ins) {
        if (v.size() != t) HEC_FAIL(HEC_ELAYOUT, "images of one batch differ in shard count");
        all.insert(all.end(), v.begin(), v.end());
        Lk.maps.insert(Lk.maps.end(), L.maps.begin(), L.maps.end());
    }
    std::vector<hec_ct *> ds;
    Layout nlk;
    bool done = false;
    HEC_CHECK(downsample_multi(c, all, Lk, select, ds, nlk, &done, mode == 2));
    if (!done) {
        for (size_t r = 0; r < ins.size(); r++) HEC_CHECK(downsample_and_merge(c, ins[r], L, select, mode, outs[r], ol));
        return HEC_OK;
    }
    Layout nl = nlk;
    nl.maps.assign(nlk.maps.begin(), nlk.maps.begin() + t);
    hec_status s = HEC_OK;
    for (size_t r = 0; r < ins.size(); r++) {
        std::vector<hec_ct *> mine(ds.begin() + r * t, ds.begin() + (r + 1) * t);
        for (size_t i = 0; i < t; i++) ds[r * t + i] = nullptr;
        if (s == HEC_OK) s = merge_downsampled(c, mine, nl, outs[r], ol);
        else free_all(mine);
    }
    if (s != HEC_OK)
        for (auto &v : outs) free_all(v);
    return s;
}

static hec_status downsample_and_merge(hec_ctx *c, const std::vector<hec_ct *> &in, const Layout &L, bool select,
                                       int mode, std::vector<hec_ct *> &out, Layout &ol)
{
    std::vector<hec_ct *> ds;
    if (L.channel) {
        HEC_CHECK(downsample_channel(c, in, L, select, mode == 4 ? 0 : mode, ds));
        const uint32_t H2 = select ? (L.H + 1) / 2 : L.H / 2, W2 = select ? (L.W + 1) / 2 : L.W / 2;
        hec_status s = merge_channel(c, ds, L, H2, W2, out, ol);
        free_all(ds);
        return s;
    }
    Layout nl;
    bool done = false;
    // modes 4 and 2: the stages of all image shards together (mode 2 for more than one shard)
    if (mode == 4 || (mode == 2 && in.size() > 1))
        HEC_CHECK(downsample_multi(c, in, L, select, ds, nl, &done, mode == 2));
    if (!done) HEC_CHECK(downsample(c, in, L, select, mode == 4 ? 0 : mode, ds, nl));
    return merge_downsampled(c, ds, nl, out, ol);
}

// rotation steps of a pooling step (for key generation)
void pool_steps(const Layout &L, bool select, uint32_t level, std::set<int32_t> &steps)
{
    const uint32_t mp = L.mp;
    uint32_t Ho = select ? (L.H + 1) / 2 : L.H / 2, Wo = select ? (L.W + 1) / 2 : L.W / 2;
    if (!select) { steps.insert(1); steps.insert((int32_t)mp); steps.insert((int32_t)mp + 1); }
    for (uint32_t i = 1; i < Wo; i++) steps.insert((int32_t)i);
    for (uint32_t j = 1; j < Ho; j++) steps.insert((int32_t)(3 * j * mp / 2));
    (void)level;
    const uint32_t N = L.N;
    auto neg = [&](int64_t a) { int64_t r = (-a) % (int64_t)N; return (int32_t)(r < 0 ? r + N : r); };
    if (L.channel) {
        // vertical shifts of every local pooled row; consolidation by N/4; duplication by N/2
        for (uint32_t j = 1; j < L.R() / 2; j++) steps.insert((int32_t)(3 * j * mp / 2));
        const size_t t = L.cs.size();
        for (uint32_t e = 1; e < (t >= 4 ? 4u : (uint32_t)t); e++) steps.insert(neg((int64_t)e * (N / 4)));
        if (t == 2) steps.insert(neg(N / 2));
        return;
    }
    const uint32_t Bn = L.B() / 4, t = (uint32_t)L.maps.size();
    if (t == 1) for (uint32_t m = 1; m < 4; m++) steps.insert(neg((int64_t)m * Bn));
    else {
        uint32_t g = t >= 4 ? 4 : t;  // the first group is the largest
        for (uint32_t e = 1; e < g; e++) steps.insert(neg((int64_t)e * Bn));
        if (t == 2) steps.insert(neg(2 * (int64_t)Bn));
    }
}

// ---------------------------------------------------------------------------
// conv plans
// ---------------------------------------------------------------------------
struct hec_conv_plan {
    hec_ctx *ctx = nullptr;
    Layout in, out;  // out = unstrided output layout
    uint32_t level = 0, stride = 1;
    int mode = 0;
    int ds_mode = -1;  // form of the stride-2 downsampling (-1: the plan mode's own)
    bool q_only = false;  // weight plaintexts over Q only: modes 0 and 1
    // basis-mask form (basis = s > 0): the plaintexts of items are borrowed
    // handles on weight rows of Wt (the nb integers round(w_b q_l / 2^s), as
    // int64_t), E the tap masks per block at 2^s
    uint32_t basis = 0, nbasis = 0;
    u64 *E = nullptr, *Wt = nullptr;
    typedef RotTerm Item;
    std::vector<std::vector<Item>> items;  // per input shard
    std::set<int32_t> steps;
    // what the baby-step / giant-step form is rebuilt from
    std::vector<double> w;
    uint32_t Co = 0, kh = 0, kw = 0, pad = 0;
    // baby-step / giant-step form, built on the first switch to mode 3: per
    // input shard one term per baby (block offset) whose products go into the
    // sums T_k, k -> (giant, output shard) = gv[k]
    bool bsgs_ready = false;
    std::vector<std::pair<int32_t, uint32_t>> gv;
    std::vector<std::vector<RotTerm>> bsgs;
};

extern "C" void he_conv2d_plan_free(hec_conv_plan *p)
{
    if (!p) return;
    for (auto *set : {&p->items, &p->bsgs})
        for (auto &v : *set)
            for (auto &it : v)
                for (auto &pp : it.pts) pt_free(pp.second);
    p->ctx->release(p->E);
    p->ctx->release(p->Wt);
    delete p;
}

static bool same_layout(const Layout &a, const Layout &b)
{
    return a.N == b.N && a.C == b.C && a.H == b.H && a.W == b.W && a.mp == b.mp && a.maps == b.maps &&
           a.channel == b.channel && a.cs == b.cs;
}

// Baby-step / giant-step form of a plan.  pt * rot_{b+g}(ct) = rot_g(pt'' * rot_b(ct))
// with pt''[i] = pt[i - g] (the weights rotated back by the giant step), so
// that T_{g,v} = sum over inputs and babies of pt'' * rot_b(ct) needs only the
// hoisted baby rotations of each input, and output v = sum_g rot_g(T_{g,v}).
static hec_status build_bsgs(hec_ctx *c, hec_conv_plan *p)
{
    if (p->bsgs_ready) return HEC_OK;
    std::vector<std::vector<ConvItem>> items;
    Layout out;
    if (p->in.channel) HEC_CHECK(conv_items_channel(p->in, p->w.data(), p->Co, p->kh, p->kw, p->pad, out, items));
    else HEC_CHECK(conv_items(p->in, p->w.data(), p->Co, p->kh, p->kw, p->pad, out, items));
    const size_t N = c->N;
    std::map<std::pair<int32_t, uint32_t>, uint32_t> idx;
    for (auto &v : items)
        for (auto &it : v)
            for (auto &pp : it.pts) idx[{it.giant, pp.first}] = 0;
    std::vector<std::pair<int32_t, uint32_t>> gv;
    for (auto &kv : idx) {
        kv.second = (uint32_t)gv.size();
        gv.push_back(kv.first);
    }
    // per input: baby -> list of (sum index, rotated weight vector)
    std::vector<std::map<int32_t, std::vector<std::pair<uint32_t, std::vector<double>>>>> byb(items.size());
    size_t nvec = 0;
    for (size_t u = 0; u < items.size(); u++)
        for (auto &it : items[u])
            for (auto &pp : it.pts) {
                std::vector<double> r(N);
                for (size_t i = 0; i < N; i++) r[(i + (size_t)it.giant) % N] = pp.second[i];
                byb[u][it.baby].push_back({idx[{it.giant, pp.first}], std::move(r)});
                nvec++;
            }
    std::vector<const double *> zp;
    zp.reserve(nvec);
    for (auto &m : byb)
        for (auto &kv : m)
            for (auto &e : kv.second) zp.push_back(e.second.data());
    std::vector<hec_pt *> pts;
    HEC_CHECK(pt_encode_many(c, zp, N, p->level, (double)c->mod[p->level], pts, true));
    size_t q = 0;
    p->bsgs.assign(items.size(), {});
    for (size_t u = 0; u < items.size(); u++)
        for (auto &kv : byb[u]) {
            RotTerm t;
            t.amount = kv.first;
            for (auto &e : kv.second) t.pts.push_back({e.first, pts[q++]});
            p->bsgs[u].push_back(std::move(t));
        }
    p->gv = gv;
    p->bsgs_ready = true;
    return HEC_OK;
}

extern "C" hec_status he_conv2d_plan_create(hec_ctx *c, const hec_image *like, const double *w, uint32_t Co,
                                            uint32_t kh, uint32_t kw, uint32_t stride, uint32_t pad,
                                            hec_conv_plan **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !like || !w || !Co || !kh || !kw) HEC_FAIL(HEC_EINVAL, "bad convolution arguments");
    if (like->shards.empty()) HEC_FAIL(HEC_ELAYOUT, "empty image");
    const uint32_t lvl = like->shards[0]->level;
    for (auto *s : like->shards)
        if (s->level != lvl) HEC_FAIL(HEC_ELEVEL, "shards at different levels");
    return conv_plan_create(c, like->lay, lvl, w, Co, kh, kw, stride, pad, out);
}

extern "C" hec_status he_conv2d_plan_create_ex(hec_ctx *c, const hec_image *like, const double *w, uint32_t Co,
                                               uint32_t kh, uint32_t kw, uint32_t stride, uint32_t pad,
                                               uint32_t flags, hec_conv_plan **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !like || !w || !Co || !kh || !kw) HEC_FAIL(HEC_EINVAL, "bad convolution arguments");
    if (flags & ~(uint32_t)(HEC_PLAN_Q_ONLY | HEC_PLAN_BASIS | HEC_PLAN_BASIS_SCALE(0xffu)))
        HEC_FAIL(HEC_EINVAL, "unknown plan flags");
    const uint32_t bs = (flags >> 8) & 0xffu;
    if ((flags & HEC_PLAN_BASIS) && (bs < 1 || bs > 50))
        HEC_FAIL(HEC_EINVAL, "basis-mask plan needs a mask scale 2^s with 1 <= s <= 50");
    if (!(flags & HEC_PLAN_BASIS) && bs) HEC_FAIL(HEC_EINVAL, "mask scale without HEC_PLAN_BASIS");
    if ((flags & HEC_PLAN_BASIS) && (flags & HEC_PLAN_Q_ONLY))
        HEC_FAIL(HEC_EINVAL, "HEC_PLAN_BASIS and HEC_PLAN_Q_ONLY exclude each other");
    if (like->shards.empty()) HEC_FAIL(HEC_ELAYOUT, "empty image");
    const uint32_t lvl = like->shards[0]->level;
    for (auto *s : like->shards)
        if (s->level != lvl) HEC_FAIL(HEC_ELEVEL, "shards at different levels");
    return conv_plan_create(c, like->lay, lvl, w, Co, kh, kw, stride, pad, out, (flags & HEC_PLAN_Q_ONLY) != 0,
                            (flags & HEC_PLAN_BASIS) ? bs : 0);
}

// The basis-mask form of a plan's weight plaintexts: per tap and block the
// mask of the tap restricted to the block, encoded at 2^s over Q_l and P
// (E, [taps][nb][nqp][n]); per (item, output) a weight row of the nb integers
// round_half_away(w_b * q_l / 2^s) (0 for blocks without a weight); each
// item's plaintexts become borrowed handles on their rows.
// sum_b round(w_b q_l / 2^s) * E_b is then the plaintext, exactly.  The
// product kernels take the weights as signed 32-bit factors and offset their
// sums by q * 2^62: |w^| < 2^31 and every prime >= 2^36 are required.
static hec_status build_basis(hec_ctx *c, hec_conv_plan *p, const std::vector<std::vector<ConvItem>> &items,
                              uint32_t s)
{
    const Layout &L = p->in;
    const uint32_t lvl = p->level, N = c->N, B = L.B(), nb = L.nb(), ntap = p->kh * p->kw;
    const uint32_t nq = lvl + 1, nqp = nq + c->k;
    const size_t n = c->n;
    const int Ho = (int)L.H + 2 * (int)p->pad - (int)p->kh + 1, Wo = (int)L.W + 2 * (int)p->pad - (int)p->kw + 1;
    // basis polynomials
    std::vector<std::vector<double>> zs;
    std::vector<const double *> zp;
    std::vector<double> mask;
    for (uint32_t t = 0; t < ntap; t++) {
        bool any;
        tap_mask(L, Ho, Wo, (int)(t / p->kw) - (int)p->pad, (int)(t % p->kw) - (int)p->pad, mask, any);
        for (uint32_t b = 0; b < nb; b++) {
            std::vector<double> z(N, 0.0);
            std::copy(mask.begin(), mask.begin() + B, z.begin() + (size_t)b * B);
            zs.push_back(std::move(z));
        }
    }
    for (auto &z : zs) zp.push_back(z.data());
    std::vector<hec_pt *> bp;
    HEC_CHECK(pt_encode_many(c, zp, N, lvl, std::ldexp(1.0, (int)s), bp, true));
    p->E = c->alloc(zs.size() * nqp * n);
    hec_status st = p->E ? HEC_OK : HEC_ENOMEM;
    for (size_t i = 0; i < bp.size() && st == HEC_OK; i++)
        if (hipMemcpyAsync(p->E + i * nqp * n, bp[i]->d, nqp * n * 8, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
            st = HEC_EDEVICE;
    for (auto *q : bp) pt_free(q);
    if (st != HEC_OK) HEC_FAIL(st, "basis polynomial storage");
    // weight rows
    for (uint32_t i = 0; i < nqp; i++)
        if (c->mod[i < nq ? i : c->L + 1 + (i - nq)] < (1ull << 36))
            HEC_FAIL(HEC_EINVAL, "basis-mask plaintexts need primes of at least 37 bits");
    const double wscale = (double)c->mod[lvl] / std::ldexp(1.0, (int)s);
    size_t rows = 0;
    for (auto &v : items)
        for (auto &it : v) rows += it.pts.size();
    std::vector<int64_t> hw(rows * nb, 0);
    size_t r = 0;
    for (auto &v : items)
        for (auto &it : v)
            for (size_t e = 0; e < it.pts.size(); e++, r++)
                for (auto &bw : it.bw[e]) {
                    int64_t wh;
                    HEC_CHECK(const_coeff(bw.second, wscale, &wh));
                    if (wh >= (1ll << 31) || wh <= -(1ll << 31))
                        HEC_FAIL(HEC_EINVAL, "weight %g too large for basis-mask plaintexts at 2^%u (|w q_l / 2^s| must "
                                 "stay below 2^31)", bw.second, s);
                    hw[(size_t)r * nb + bw.first] = wh;
                }
    p->Wt = c->alloc(hw.size());
    if (!p->Wt) HEC_FAIL(HEC_ENOMEM, "weight rows");
    HEC_TRY_HIP(hipMemcpyAsync(p->Wt, hw.data(), hw.size() * 8, hipMemcpyHostToDevice, c->st));
    HEC_TRY_HIP(hipStreamSynchronize(c->st));
    p->basis = s;
    p->nbasis = nb;
    return HEC_OK;
}

const Layout &conv_plan_out(const hec_conv_plan *p) { return p->out; }

hec_status conv_plan_create(hec_ctx *c, const Layout &lay, uint32_t lvl, const double *w, uint32_t Co, uint32_t kh,
                            uint32_t kw, uint32_t stride, uint32_t pad, hec_conv_plan **out, bool q_only,
                            uint32_t basis)
{
    *out = nullptr;
    if (!w || !Co || !kh || !kw) HEC_FAIL(HEC_EINVAL, "bad convolution arguments");
    if (stride != 1 && stride != 2) HEC_FAIL(HEC_EINVAL, "stride must be 1 or 2");
    if (!lay.shards()) HEC_FAIL(HEC_ELAYOUT, "empty image");
    if (lvl < 1) HEC_FAIL(HEC_ELEVEL, "convolution needs a level");
    if (stride == 2 && lvl < 2) HEC_FAIL(HEC_ELEVEL, "strided convolution needs two levels");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    std::unique_ptr<hec_conv_plan> p(new hec_conv_plan());
    p->ctx = c;
    p->in = lay;
    p->level = lvl;
    p->stride = stride;
    std::vector<std::vector<ConvItem>> items;
    if (lay.channel) HEC_CHECK(conv_items_channel(lay, w, Co, kh, kw, pad, p->out, items));
    else HEC_CHECK(conv_items(lay, w, Co, kh, kw, pad, p->out, items));
    p->items.resize(items.size());
    p->w.assign(w, w + (size_t)Co * lay.C * kh * kw);
    p->Co = Co;
    p->kh = kh;
    p->kw = kw;
    p->pad = pad;
    std::vector<hec_pt *> pts;
    p->q_only = q_only;
    if (basis) {
        if (lay.channel) HEC_FAIL(HEC_ELAYOUT, "basis-mask plaintexts need an image-sharded input");
        if (lay.nb() > HEC_BASIS_NB)
            HEC_FAIL(HEC_ELAYOUT, "basis-mask plaintexts take at most %d blocks per shard (layout has %u)",
                     HEC_BASIS_NB, lay.nb());
        if (hec_status bs = build_basis(c, p.get(), items, basis)) {
            c->release(p->E);
            c->release(p->Wt);
            return bs;
        }
        size_t r = 0;
        for (auto &v : items)
            for (auto &it : v)
                for (size_t e = 0; e < it.pts.size(); e++, r++) {
                    hec_pt *h = new hec_pt();
                    h->ctx = c;
                    h->level = lvl;
                    h->scale = (double)c->mod[lvl];
                    h->d = p->Wt + r * p->nbasis;
                    h->has_p = true;
                    h->borrowed = true;
                    pts.push_back(h);
                }
    } else {
        std::vector<const double *> zp;
        for (auto &v : items)
            for (auto &it : v)
                for (auto &pp : it.pts) zp.push_back(pp.second.data());
        // limbs over Q_l and P: the lazy-ModDown mode multiplies before ModDown (over Q_l only for a plan that
        // runs per rotation, a quarter less memory)
        HEC_CHECK(pt_encode_many(c, zp, c->N, lvl, (double)c->mod[lvl], pts, !q_only));
    }
    size_t q = 0;
    for (size_t u = 0; u < items.size(); u++)
        for (auto &it : items[u]) {
            hec_conv_plan::Item pi;
            pi.amount = it.amount;
            pi.tap = basis ? it.tap : -1;
            for (auto &pp : it.pts) pi.pts.push_back({pp.first, pts[q++]});
            // keys for every mode: the amounts, and their baby and giant parts
            for (int32_t a : {it.amount, it.baby, it.giant})
                if (a % (int32_t)c->N) p->steps.insert(a);
            p->items[u].push_back(std::move(pi));
        }
    if (stride == 2) {
        Layout o = p->out;
        pool_steps(o, true, lvl - 1, p->steps);
    }
    *out = p.release();
    return HEC_OK;
}

extern "C" hec_status he_conv2d_plan_set_mode(hec_conv_plan *p, int mode)
{
    if (!p || mode < 0 || mode > 4) HEC_FAIL(HEC_EINVAL, "bad mode");
    if (p->q_only && (mode == 2 || mode == 3))
        HEC_FAIL(HEC_EINVAL, "plan without special-prime limbs runs in modes 0, 1 and 4 only");
    if (p->basis && mode == 3) HEC_FAIL(HEC_EINVAL, "basis-mask plan runs in modes 0, 1 and 2");
    if (mode == 3) {
        HEC_TRY_HIP(hipSetDevice(p->ctx->dev));
        HEC_CHECK(build_bsgs(p->ctx, p));
    }
    p->mode = mode;
    return HEC_OK;
}

extern "C" hec_status he_conv2d_plan_set_downsample_mode(hec_conv_plan *p, int mode)
{
    if (!p) HEC_FAIL(HEC_EINVAL, "plan is NULL");
    if (p->stride != 2) HEC_FAIL(HEC_EINVAL, "a stride-1 plan has no downsampling step");
    if (mode != -1 && mode != 0 && mode != 2 && mode != 4)
        HEC_FAIL(HEC_EINVAL, "downsampling mode must be -1, 0, 2 or 4");
    p->ds_mode = mode;
    return HEC_OK;
}

extern "C" hec_status he_conv2d_plan_steps(const hec_conv_plan *p, int32_t *steps, size_t cap, size_t *count)
{
    if (!p) HEC_FAIL(HEC_EINVAL, "plan is NULL");
    if (count) *count = p->steps.size();
    if (steps) {
        if (cap < p->steps.size()) HEC_FAIL(HEC_EINVAL, "capacity too small");
        size_t i = 0;
        for (int32_t s : p->steps) steps[i++] = s;
    }
    return HEC_OK;
}

// acc[v] (+)= sum over the chunk's rotations t of rots[t] * (plaintext of term
// i0 + t for v): output groups of HEC_MAC_OUTS, term batches of HEC_MAC_TERMS,
// one launch each; first[v] set: output v not written yet (cleared here)
static hec_status mac_rotations(hec_ctx *c, const std::vector<hec_ct *> &rots,
                                const std::vector<hec_conv_plan::Item> &its, size_t i0, std::vector<hec_ct *> &acc,
                                std::vector<char> &first, const BasisArg *bt)
{
    const size_t nout = acc.size(), cnt = rots.size();
    const uint32_t lvl = rots[0]->level;
    for (size_t t = 0; t < cnt; t++)
        for (auto &pp : its[i0 + t].pts)
            if (pp.second->level != lvl || rots[t]->level != lvl || acc[pp.first]->level != lvl)
                HEC_FAIL(HEC_ELEVEL, "level mismatch in pt product");
    for (size_t v0 = 0; v0 < nout; v0 += HEC_MAC_OUTS) {
        const size_t nv = std::min((size_t)HEC_MAC_OUTS, nout - v0);
        for (size_t t0 = 0; t0 < cnt; t0 += HEC_MAC_TERMS) {
            const size_t nt = std::min((size_t)HEC_MAC_TERMS, cnt - t0);
            MacBatch b{};
            BasisArg ba = bt ? *bt : BasisArg{};
            bool any = false;
            for (size_t t = 0; t < nt; t++) {
                b.ct[t] = rots[t0 + t]->d;
                if (bt) {
                    if (its[i0 + t0 + t].tap < 0) HEC_FAIL(HEC_EINVAL, "basis-mask term without a tap");
                    ba.tap[t] = (u32)its[i0 + t0 + t].tap;
                }
                for (auto &pp : its[i0 + t0 + t].pts)
                    if (pp.first >= v0 && pp.first < v0 + nv) {
                        b.pt[t][pp.first - v0] = pp.second->d;
                        any = true;
                    }
            }
            if (!any) continue;
            int fbits = 0;
            for (size_t j = 0; j < nv; j++) {
                bool used = false;
                for (size_t t = 0; t < nt && !used; t++) used = b.pt[t][j] != nullptr;
                if (!used) continue;
                b.out[j] = acc[v0 + j]->d;
                if (first[v0 + j]) {
                    fbits |= 1 << j;
                    first[v0 + j] = 0;
                    for (size_t t = 0; t < nt; t++)
                        if (b.pt[t][j]) {
                            acc[v0 + j]->scale = rots[t0 + t]->scale * its[i0 + t0 + t].pts[0].second->scale;
                            break;
                        }
                }
            }
            if (!hec_mac_terms(c->T, b, (int)nt, (int)nv, (int)lvl + 1, fbits, c->st, bt ? &ba : nullptr))
                HEC_FAIL(HEC_EINVAL, "invalid plaintext-product batch");
        }
    }
    return HEC_OK;
}

// Plan mode 4: the products of mode 0 with the rotations of all input shards
// taken together amount by amount (ct_rotate_multi: each rotation key read
// once for the shards of a group of up to 64 instead of once per shard), the
// zero rotations straight from the inputs.  Every rotation and every sum is
// the one mode 0 computes, so the ciphertexts are mode 0's bit for bit.
static hec_status conv_key_stationary(hec_ctx *c, const std::vector<const hec_ct *> &ins,
                                      const std::vector<std::vector<hec_conv_plan::Item>> &items,
                                      std::vector<hec_ct *> &acc, std::vector<char> &first, const BasisArg *bt)
{
    typedef hec_conv_plan::Item Item;
    std::vector<hec_ct *> zr;
    std::vector<Item> zi;
    for (size_t u = 0; u < ins.size(); u++)
        for (const Item &it : items[u])
            if (c->galois(it.amount) == 1) {
                zr.push_back(const_cast<hec_ct *>(ins[u]));
                zi.push_back(it);
            }
    if (!zr.empty()) HEC_CHECK(mac_rotations(c, zr, zi, 0, acc, first, bt));
    for (size_t u0 = 0; u0 < ins.size(); u0 += HEC_MULTI_MAX_INPUTS) {
        const size_t S = std::min((size_t)HEC_MULTI_MAX_INPUTS, ins.size() - u0);
        std::vector<const hec_ct *> grp(ins.begin() + u0, ins.begin() + u0 + S);
        // amounts in first-use order; per (amount, shard) the items that rotate by it
        std::vector<int32_t> amounts;
        std::vector<uint64_t> want;
        std::map<int32_t, size_t> idx;
        std::vector<std::vector<std::vector<const Item *>>> by;  // [amount][shard]
        for (size_t u = 0; u < S; u++)
            for (const Item &it : items[u0 + u]) {
                if (c->galois(it.amount) == 1) continue;
                auto f = idx.find(it.amount);
                size_t a;
                if (f == idx.end()) {
                    a = amounts.size();
                    idx[it.amount] = a;
                    amounts.push_back(it.amount);
                    want.push_back(0);
                    by.emplace_back(S);
                } else {
                    a = f->second;
                }
                want[a] |= 1ull << u;
                by[a][u].push_back(&it);
            }
        auto sink = [&](size_t a0, size_t na, const std::vector<hec_ct *> &rots) -> hec_status {
            std::vector<hec_ct *> rs;
            std::vector<Item> its;
            for (size_t t = 0; t < na; t++)
                for (size_t u = 0; u < S; u++)
                    for (const Item *it : by[a0 + t][u]) {
                        rs.push_back(rots[t * S + u]);
                        its.push_back(*it);
                    }
            return rs.empty() ? HEC_OK : mac_rotations(c, rs, its, 0, acc, first, bt);
        };
        HEC_CHECK(ct_rotate_multi(c, grp, amounts, want, (size_t)hec_tune_params().ks_amounts, sink));
    }
    return HEC_OK;
}

#define ROT_CHUNK 32
extern "C" hec_status he_conv2d_plan_run(hec_ctx *c, const hec_conv_plan *p, const hec_image *in, hec_image **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !p || !in) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (!same_layout(p->in, in->lay)) HEC_FAIL(HEC_ELAYOUT, "image layout differs from the plan's");
    for (auto *s : in->shards)
        if (s->level != p->level) HEC_FAIL(HEC_ELEVEL, "image level differs from the plan's");
    for (int32_t s : p->steps)
        if (!have_rotkey(c, s)) HEC_FAIL(HEC_ENOKEY, "no rotation key for step %d", s);
    HEC_TRY_HIP(hipSetDevice(c->dev));
    const size_t nout = p->out.shards();
    std::vector<hec_ct *> acc(nout, nullptr);
    std::vector<char> first(nout, 1);
    for (size_t v = 0; v < nout; v++) {
        acc[v] = ct_new(c, p->level, 1.0);
        if (!acc[v]) { free_all(acc); HEC_FAIL(HEC_ENOMEM, "accumulator allocation"); }
    }
    hec_status s = HEC_OK;
    std::vector<const hec_ct *> ins(in->shards.begin(), in->shards.end());
    BasisArg bt{};
    if (p->basis) {
        bt.E = p->E;
        bt.nb = p->nbasis;
        bt.nqp = p->level + 1 + c->k;
    }
    const BasisArg *btp = p->basis ? &bt : nullptr;
    if (p->mode == 2) {
        free_all(acc);
        s = lazy_rotate_mac(c, ins, p->items, nout, acc, btp);
        std::fill(first.begin(), first.end(), 0);
    } else if (p->mode == 3) {
        // baby steps: T_k = sum of pt'' * rot_baby(ct_u) (one ModDown per k);
        // giant steps: output v = sum_k rot_giant(T_k) over the k of v (one more ModDown)
        free_all(acc);
        s = bsgs_eval(c, ins, p->bsgs, p->gv, nout, acc);
        std::fill(first.begin(), first.end(), 0);
    } else if (p->mode == 4) {
        s = conv_key_stationary(c, ins, p->items, acc, first, btp);
    }
    for (size_t u = 0; u < p->items.size() && s == HEC_OK && p->mode < 2; u++) {
        const auto &its = p->items[u];
        // mode 0: one ModUp of the shard for all its chunks of rotations
        u64 *Du = nullptr;
        if (p->mode == 0) {
            bool any = false;
            for (const auto &it : its) any = any || c->galois(it.amount) != 1;
            if (any) s = ct_modup(c, in->shards[u], &Du);
        }
        for (size_t i0 = 0; i0 < its.size() && s == HEC_OK; i0 += ROT_CHUNK) {
            size_t cnt = std::min((size_t)ROT_CHUNK, its.size() - i0);
            std::vector<int32_t> st(cnt);
            for (size_t t = 0; t < cnt; t++) st[t] = its[i0 + t].amount;
            std::vector<hec_ct *> rots(cnt, nullptr);
            if (p->mode == 0) {
                s = ct_rotate_hoisted(c, in->shards[u], st.data(), cnt, rots.data(), Du);
            } else {
                for (size_t t = 0; t < cnt && s == HEC_OK; t++) s = ckks_rotate(c, in->shards[u], st[t], &rots[t]);
            }
            if (s == HEC_OK) s = mac_rotations(c, rots, its, i0, acc, first, btp);
            free_all(rots);
        }
        c->release(Du);
    }
    for (size_t v = 0; v < nout && s == HEC_OK; v++) {
        if (first[v]) s = HEC_ELAYOUT, hec_set_error("output shard %zu received no product", v);
        else s = ct_rescale(c, acc[v]);
    }
    if (s != HEC_OK) { free_all(acc); return s; }
    hec_image *im = new hec_image();
    im->ctx = c;
    if (p->stride == 1) {
        im->lay = p->out;
        im->shards = acc;
    } else {
        const int dm = p->ds_mode >= 0 ? p->ds_mode : (p->mode == 1 ? 0 : p->mode);
        s = downsample_and_merge(c, acc, p->out, true, dm, im->shards, im->lay);
        free_all(acc);
        if (s != HEC_OK) { hec_image_free(im); return s; }
    }
    *out = im;
    return HEC_OK;
}

// Several images of a plan's layout and level in one evaluation (a server's
// batch of requests): in mode 4 the rotations of all shards of all images go
// through the key switch together amount by amount (each key read once per
// group of up to 64 shards of the whole batch) and the stride-2 downsampling
// stages likewise; other modes run image by image.  Same ciphertexts as one
// he_conv2d_plan_run per image.
hec_status conv_plan_run_multi(hec_ctx *c, const hec_conv_plan *p, const std::vector<const hec_image *> &ins,
                               std::vector<hec_image *> &outs)
{
    outs.assign(ins.size(), nullptr);
    auto fail = [&](hec_status s) {
        for (auto *&im : outs) {
            hec_image_free(im);
            im = nullptr;
        }
        return s;
    };
    if (p->mode != 4 || ins.size() == 1) {
        for (size_t r = 0; r < ins.size(); r++) {
            hec_status s = he_conv2d_plan_run(c, p, ins[r], &outs[r]);
            if (s != HEC_OK) return fail(s);
        }
        return HEC_OK;
    }
    for (auto *im : ins) {
        if (!same_layout(p->in, im->lay)) HEC_FAIL(HEC_ELAYOUT, "image layout differs from the plan's");
        for (auto *sh : im->shards)
            if (sh->level != p->level) HEC_FAIL(HEC_ELEVEL, "image level differs from the plan's");
    }
    for (int32_t st : p->steps)
        if (!have_rotkey(c, st)) HEC_FAIL(HEC_ENOKEY, "no rotation key for step %d", st);
    HEC_TRY_HIP(hipSetDevice(c->dev));
    const size_t nout = p->out.shards(), K = ins.size();
    std::vector<const hec_ct *> all;
    std::vector<std::vector<hec_conv_plan::Item>> items;
    for (size_t r = 0; r < K; r++)
        for (size_t u = 0; u < ins[r]->shards.size(); u++) {
            all.push_back(ins[r]->shards[u]);
            items.push_back(p->items[u]);
            for (auto &it : items.back())
                for (auto &pp : it.pts) pp.first += (uint32_t)(r * nout);
        }
    std::vector<hec_ct *> acc(K * nout, nullptr);
    std::vector<char> first(K * nout, 1);
    for (auto *&a : acc)
        if (!(a = ct_new(c, p->level, 1.0))) { free_all(acc); HEC_FAIL(HEC_ENOMEM, "accumulator allocation"); }
    BasisArg bt{};
    if (p->basis) {
        bt.E = p->E;
        bt.nb = p->nbasis;
        bt.nqp = p->level + 1 + c->k;
    }
    hec_status s = conv_key_stationary(c, all, items, acc, first, p->basis ? &bt : nullptr);
    for (size_t v = 0; v < acc.size() && s == HEC_OK; v++) {
        if (first[v]) s = HEC_ELAYOUT, hec_set_error("output shard %zu received no product", v % nout);
        else s = ct_rescale(c, acc[v]);
    }
    if (s != HEC_OK) { free_all(acc); return s; }
    std::vector<std::vector<hec_ct *>> per(K);
    for (size_t r = 0; r < K; r++) per[r].assign(acc.begin() + r * nout, acc.begin() + (r + 1) * nout);
    if (p->stride == 1) {
        for (size_t r = 0; r < K; r++) {
            outs[r] = new hec_image();
            outs[r]->ctx = c;
            outs[r]->lay = p->out;
            outs[r]->shards = per[r];
        }
        return HEC_OK;
    }
    std::vector<std::vector<hec_ct *>> ds;
    Layout ol;
    s = downsample_and_merge_multi(c, per, p->out, true, p->ds_mode >= 0 ? p->ds_mode : 4, ds, ol);
    free_all(acc);
    if (s != HEC_OK) return s;
    for (size_t r = 0; r < K; r++) {
        outs[r] = new hec_image();
        outs[r]->ctx = c;
        outs[r]->lay = ol;
        outs[r]->shards = ds[r];
    }
    return HEC_OK;
}

// 2x2 average pooling of several images of one layout (he_avgpool_ex per
// image; mode 4 takes the stages of all images' shards together)
hec_status avgpool_multi(hec_ctx *c, const std::vector<const hec_image *> &ins, int mode,
                         std::vector<hec_image *> &outs)
{
    outs.assign(ins.size(), nullptr);
    if (ins.empty()) return HEC_OK;
    const Layout &L = ins[0]->lay;
    std::set<int32_t> steps;
    for (auto *im : ins) {
        if (!same_layout(L, im->lay)) HEC_FAIL(HEC_ELAYOUT, "images of one pooling batch differ in layout");
        if (im->shards.empty()) HEC_FAIL(HEC_ELAYOUT, "empty image");
    }
    pool_steps(L, false, ins[0]->shards[0]->level, steps);
    for (int32_t st : steps)
        if (!have_rotkey(c, st)) HEC_FAIL(HEC_ENOKEY, "no rotation key for step %d", st);
    std::vector<std::vector<hec_ct *>> in(ins.size()), ds;
    for (size_t r = 0; r < ins.size(); r++) in[r] = ins[r]->shards;
    Layout ol;
    HEC_CHECK(downsample_and_merge_multi(c, in, L, false, mode, ds, ol));
    for (size_t r = 0; r < ins.size(); r++) {
        outs[r] = new hec_image();
        outs[r]->ctx = c;
        outs[r]->lay = ol;
        outs[r]->shards = ds[r];
    }
    return HEC_OK;
}

extern "C" hec_status he_conv2d_sharded(hec_ctx *c, const hec_image *in, const double *w, uint32_t Co, uint32_t kh,
                                        uint32_t kw, uint32_t stride, uint32_t pad, const double *bias,
                                        hec_image **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    hec_conv_plan *p = nullptr;
    HEC_CHECK(he_conv2d_plan_create(c, in, w, Co, kh, kw, stride, pad, &p));
    hec_image *conv = nullptr;
    hec_status s = he_conv2d_plan_run(c, p, in, &conv);
    he_conv2d_plan_free(p);
    if (s != HEC_OK || !bias) {
        *out = conv;
        return s;
    }
    // the shift of a folded batch norm: one plaintext per output shard at the
    // output's level and scale (after the downsampling of a strided
    // convolution, which only selects pixels)
    s = he_image_add_bias(c, conv, bias, out);
    hec_image_free(conv);
    return s;
}

extern "C" hec_status he_avgpool(hec_ctx *c, const hec_image *in, uint32_t window, hec_image **out)
{
    return he_avgpool_ex(c, in, window, 0, out);
}

extern "C" hec_status he_avgpool_ex(hec_ctx *c, const hec_image *in, uint32_t window, int mode, hec_image **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !in) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (mode != 0 && mode != 2 && mode != 3 && mode != 4)
        HEC_FAIL(HEC_EINVAL, "pooling mode must be 0 (per rotation), 2 (lazy ModDown), 3 (baby-step/giant-step) "
                             "or 4 (key-stationary over the shards)");
    if (window != 2) HEC_FAIL(HEC_EINVAL, "only 2x2 pooling is supported");
    if (in->shards.empty()) HEC_FAIL(HEC_ELAYOUT, "empty image");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    std::set<int32_t> steps;
    pool_steps(in->lay, false, in->shards[0]->level, steps);
    for (int32_t s : steps)
        if (!have_rotkey(c, s)) HEC_FAIL(HEC_ENOKEY, "no rotation key for step %d", s);
    hec_image *im = new hec_image();
    im->ctx = c;
    hec_status s = downsample_and_merge(c, in->shards, in->lay, false, mode, im->shards, im->lay);
    if (s != HEC_OK) { hec_image_free(im); return s; }
    *out = im;
    return HEC_OK;
}

extern "C" hec_status he_avgpool_steps(hec_ctx *c, const hec_image *like, int32_t *steps, size_t cap, size_t *count)
{
    if (!c || !like || like->shards.empty()) HEC_FAIL(HEC_EINVAL, "bad arguments");
    std::set<int32_t> st;
    pool_steps(like->lay, false, like->shards[0]->level, st);
    if (count) *count = st.size();
    if (steps) {
        if (cap < st.size()) HEC_FAIL(HEC_EINVAL, "capacity too small");
        size_t i = 0;
        for (int32_t x : st) steps[i++] = x;
    }
    return HEC_OK;
}

// ---------------------------------------------------------------------------
// linear and pool-linear layers (Section 4.3, "Linear")
// ---------------------------------------------------------------------------
// Slot vectors of the weights: vec[o][u] multiplies shard u for output o
// (empty = zero).  Linear: W is [O][C*H*W] over the input in [C][H][W] order;
// pool-linear: W is [O][C], and every valid position of channel f carries
// W[o][f] / (H*W).  A channel held in several blocks is read from its first
// block in shard-then-block order only.
static hec_status linear_vectors(const Layout &L, const double *W, uint32_t O, bool pool,
                                 std::vector<std::vector<std::vector<double>>> &vec)
{
    const uint32_t C = L.C, H = L.H, Wd = L.W, N = L.N, mp = L.mp;
    auto weight = [&](uint32_t o, uint32_t f, uint32_t i, uint32_t j) {
        return pool ? W[(size_t)o * C + f] / (double)(H * Wd) : W[(((size_t)o * C + f) * H + i) * Wd + j];
    };
    vec.assign(O, std::vector<std::vector<double>>(L.shards()));
    if (L.channel) {
        const uint32_t R = L.R();
        for (size_t u = 0; u < L.cs.size(); u++) {
            const uint32_t f = (uint32_t)L.cs[u].first, part = (uint32_t)L.cs[u].second;
            if (part * R >= H) continue;
            for (uint32_t o = 0; o < O; o++) {
                std::vector<double> v(N, 0.0);
                for (uint32_t r = 0; r < R && part * R + r < H; r++)
                    for (uint32_t j = 0; j < Wd; j++) v[(size_t)r * mp + j] = weight(o, f, part * R + r, j);
                vec[o][u] = std::move(v);
            }
        }
        return HEC_OK;
    }
    std::vector<char> seen(C, 0);
    std::vector<std::pair<uint32_t, uint32_t>> place;  // (shard, block) per first occurrence
    std::vector<uint32_t> chan;
    for (uint32_t u = 0; u < L.maps.size(); u++)
        for (uint32_t b = 0; b < L.nb(); b++) {
            const int32_t f = L.maps[u][b];
            if (f >= 0 && !seen[f]) {
                seen[f] = 1;
                place.push_back({u, b});
                chan.push_back((uint32_t)f);
            }
        }
    if (place.size() != C) HEC_FAIL(HEC_ELAYOUT, "channel missing from the layout");
    for (uint32_t o = 0; o < O; o++)
        for (size_t t = 0; t < place.size(); t++) {
            auto &v = vec[o][place[t].first];
            if (v.empty()) v.assign(N, 0.0);
            const size_t base = (size_t)place[t].second * L.B();
            for (uint32_t i = 0; i < H; i++)
                for (uint32_t j = 0; j < Wd; j++) v[base + (size_t)i * mp + j] = weight(o, chan[t], i, j);
        }
    return HEC_OK;
}

extern "C" hec_status he_linear_steps(hec_ctx *c, const hec_image *like, int32_t *steps, size_t cap, size_t *count)
{
    if (!c || !like) HEC_FAIL(HEC_EINVAL, "NULL argument");
    std::vector<int32_t> st;
    for (uint32_t k = c->N / 2; k >= 1; k /= 2) st.push_back((int32_t)k);
    if (count) *count = st.size();
    if (steps) {
        if (cap < st.size()) HEC_FAIL(HEC_EINVAL, "capacity too small");
        for (size_t i = 0; i < st.size(); i++) steps[i] = st[i];
    }
    return HEC_OK;
}

extern "C" hec_status he_linear(hec_ctx *c, const hec_image *in, const double *W, uint32_t O, int pool, hec_ct **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !in || !W || !O) HEC_FAIL(HEC_EINVAL, "bad linear arguments");
    if (O > c->N) HEC_FAIL(HEC_EINVAL, "more outputs than slots");
    if (in->shards.empty()) HEC_FAIL(HEC_ELAYOUT, "empty image");
    const uint32_t lvl = in->shards[0]->level;
    for (auto *s : in->shards)
        if (s->level != lvl || s->scale != in->shards[0]->scale) HEC_FAIL(HEC_ELEVEL, "shards at different levels");
    if (lvl < 2) HEC_FAIL(HEC_ELEVEL, "the linear layer needs two levels");
    for (uint32_t k = c->N / 2; k >= 1; k /= 2)
        if (!have_rotkey(c, (int32_t)k)) HEC_FAIL(HEC_ENOKEY, "no rotation key for step %u", k);
    HEC_TRY_HIP(hipSetDevice(c->dev));
    std::vector<std::vector<std::vector<double>>> vec;
    HEC_CHECK(linear_vectors(in->lay, W, O, pool != 0, vec));
    // weight plaintexts at scale q_l, one-hot masks at scale q_{l-1}
    std::vector<const double *> zp;
    std::vector<std::pair<uint32_t, uint32_t>> which;
    for (uint32_t o = 0; o < O; o++)
        for (uint32_t u = 0; u < vec[o].size(); u++)
            if (!vec[o][u].empty()) {
                zp.push_back(vec[o][u].data());
                which.push_back({o, u});
            }
    std::vector<hec_pt *> wpts, mpts;
    HEC_CHECK(pt_encode_many(c, zp, c->N, lvl, (double)c->mod[lvl], wpts));
    std::vector<std::vector<double>> onehot(O, std::vector<double>(c->N, 0.0));
    std::vector<const double *> mz;
    for (uint32_t o = 0; o < O; o++) {
        onehot[o][o] = 1.0;
        mz.push_back(onehot[o].data());
    }
    hec_status s = pt_encode_many(c, mz, c->N, lvl - 1, (double)c->mod[lvl - 1], mpts);
    hec_ct *res = nullptr;
    size_t w = 0;
    // per output: the products summed over the shards, rescaled
    std::vector<hec_ct *> acc(O, nullptr);
    for (uint32_t o = 0; o < O && s == HEC_OK; o++) {
        acc[o] = ct_new(c, lvl, 1.0);
        if (!acc[o]) { s = HEC_ENOMEM; hec_set_error("ciphertext allocation"); break; }
        bool first = true;
        for (; w < which.size() && which[w].first == o && s == HEC_OK; w++) {
            s = ct_mac_pt(c, acc[o], in->shards[which[w].second], wpts[w], first);
            first = false;
        }
        if (s == HEC_OK && first) s = HEC_ELAYOUT, hec_set_error("output %u has no weights", o);
        if (s == HEC_OK) s = ct_rescale(c, acc[o]);
    }
    // rotate-and-add over all slots, every slot ending with its dot product;
    // the O sums rotate together, one batched key switch per step
    for (uint32_t k = c->N / 2; k >= 1 && s == HEC_OK; k /= 2) {
        std::vector<hec_ct *> rots;
        s = ct_rotate_many(c, std::vector<const hec_ct *>(acc.begin(), acc.end()), (int32_t)k, rots);
        for (uint32_t o = 0; o < O && s == HEC_OK; o++) s = ct_add_inplace(c, acc[o], rots[o]);
        free_all(rots);
    }
    for (uint32_t o = 0; o < O && s == HEC_OK; o++) {
        hec_ct *m = ct_new(c, acc[o]->level, 1.0);
        if (!m) s = HEC_ENOMEM, hec_set_error("ciphertext allocation");
        else s = ct_mac_pt(c, m, acc[o], mpts[o], true);
        if (s == HEC_OK) s = sum_into(c, res, m);
        else ct_free(m);
    }
    free_all(acc);
    if (s == HEC_OK) s = ct_rescale(c, res);
    for (auto *p : wpts) pt_free(p);
    for (auto *p : mpts) pt_free(p);
    if (s != HEC_OK) {
        ct_free(res);
        return s;
    }
    *out = res;
    return HEC_OK;
}

// ---------------------------------------------------------------------------
// per-channel bias (batch norm's shift folded into the convolution, Section
// 4.3): the packed image whose channel f is bias[f] on every valid pixel,
// encoded at each shard's level and scale and added
// ---------------------------------------------------------------------------
hec_status image_add_bias(hec_ctx *c, const std::vector<hec_ct *> &in, const Layout &L, const double *bias,
                          std::vector<hec_ct *> &out)
{
    out.clear();
    if (in.empty()) HEC_FAIL(HEC_ELAYOUT, "empty image");
    for (auto *s : in)
        if (s->level != in[0]->level || s->scale != in[0]->scale) HEC_FAIL(HEC_ELEVEL, "shards at different levels");
    for (uint32_t f = 0; f < L.C; f++)
        if (!std::isfinite(bias[f])) HEC_FAIL(HEC_EINVAL, "bias %u not finite", f);
    std::vector<double> x((size_t)L.C * L.H * L.W);
    for (uint32_t f = 0; f < L.C; f++) std::fill(x.begin() + (size_t)f * L.H * L.W, x.begin() + (size_t)(f + 1) * L.H * L.W, bias[f]);
    std::vector<std::vector<double>> v(in.size());
    std::vector<const double *> zp;
    for (uint32_t u = 0; u < in.size(); u++) {
        pack_shard(L, x.data(), u, v[u]);
        zp.push_back(v[u].data());
    }
    std::vector<hec_pt *> pts;
    HEC_CHECK(pt_encode_many(c, zp, c->N, in[0]->level, in[0]->scale, pts));
    hec_status s = HEC_OK;
    for (size_t u = 0; u < in.size() && s == HEC_OK; u++) {
        hec_ct *o = nullptr;
        s = ct_add_pt(c, in[u], pts[u], &o);
        if (s == HEC_OK) out.push_back(o);
    }
    for (auto *p : pts) pt_free(p);
    if (s != HEC_OK) free_all(out);
    return s;
}

extern "C" hec_status he_image_add_bias(hec_ctx *c, const hec_image *in, const double *bias, hec_image **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !in || !bias) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    hec_image *im = image_new(c, in->lay);
    hec_status s = image_add_bias(c, in->shards, in->lay, bias, im->shards);
    if (s != HEC_OK) {
        hec_image_free(im);
        return s;
    }
    *out = im;
    return HEC_OK;
}
