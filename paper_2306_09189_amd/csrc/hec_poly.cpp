// hec_poly.cpp -- polynomial evaluation on ciphertexts in the Chebyshev basis
// (the GELU activation of the encrypted network, Section 4.3 and the Appendix
// on polynomial approximation), with baby-step/giant-step splitting of the
// polynomial.  The S shards of an image go through the evaluation together:
// every operation is one set of launches over all of them (they share levels,
// scales and coefficients), so the small per-ciphertext launches of a long
// dependency chain become S times larger.
//
// Map: y = (2x - a - b)/(b - a) costs one constant product, except on
// [a, b] = [-1, 1], where y = x (an affine map in front of the activation
// folds into the previous convolution, as batch normalization does, so
// degree 59 takes depth 6 and degree 27 depth 5).
//
// Scale management: every ciphertext at level l carries the nominal scale
// S[l], S[l0] the input's scale and S[l-1] = S[l]^2 / q_l, so the rescaled
// product of two level-l ciphertexts has exactly S[l-1].  A constant product
// on a level-l ciphertext (or one dropped to level l) encodes the constant at
// S[l-1] q_l / (its scale) and sets the result's nominal scale to S[l-1]
// after the rescale; a level adjustment drops limbs to l+1 and multiplies by
// the constant 1 in the same way.
//
// Basis: T_1 = y, T_{2k} = 2 T_k^2 - 1, T_{2k+1} = 2 T_{k+1} T_k - T_1 for
// k < m (m the smallest power of two with m^2 >= deg + 1) and the giant
// powers T_{2m}, T_{4m}, ... by doubling.  A polynomial of degree < m is c_0
// plus the constant products c_j T_j, every T_j dropped to one level and the
// sum rescaled once; a larger one is divided by the largest giant power
// T_g <= its degree (T_j = 2 T_g T_{j-g} - T_{2g-j}), p = q T_g + r, and q, r
// are evaluated the same way.
#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <vector>

#include "hec_internal.h"

namespace {

struct Fail {
    hec_status s;
};
#define PTRY(x)                                                                                                    \
    do {                                                                                                           \
        hec_status s_ = (x);                                                                                       \
        if (s_ != HEC_OK) throw Fail{s_};                                                                          \
    } while (0)
#define PFAIL(code, ...)                                                                                           \
    do {                                                                                                           \
        hec_set_error(__VA_ARGS__);                                                                                \
        throw Fail{code};                                                                                          \
    } while (0)

// S ciphertexts at one level and nominal scale, contiguous: d = [S][2][level+1][n]
// (no device data in a dry run)
struct Batch {
    hec_ctx *c = nullptr;
    uint32_t level = 0;
    double scale = 1.0;
    u64 *d = nullptr;
    ~Batch()
    {
        if (c && d) c->release(d);
    }
};
using Ct = std::shared_ptr<Batch>;

// a ciphertext batch or a plain constant (sums of constants stay on the host)
struct Val {
    bool is_const = false;
    double c = 0.0;
    Ct ct;
    static Val constant(double v)
    {
        Val r;
        r.is_const = true;
        r.c = v;
        return r;
    }
    static Val of(Ct x)
    {
        Val r;
        r.ct = std::move(x);
        return r;
    }
};

// dry: levels and scales only, to learn the output level and check the level
// budget and constants before any launch
struct ChebEval {
    hec_ctx *c;
    Ct x;
    uint32_t S;
    double a, b;
    bool dry;
    size_t n;
    std::vector<double> S_;  // nominal scale per level

    ChebEval(hec_ctx *ctx, Ct in, uint32_t count, double lo, double hi, bool dry_run)
        : c(ctx), x(std::move(in)), S(count), a(lo), b(hi), dry(dry_run), n(ctx->n)
    {
        S_.assign(x->level + 1, 0.0);
        S_[x->level] = x->scale;
        for (uint32_t l = x->level; l > 0; l--) S_[l - 1] = (S_[l] * S_[l]) / (double)c->mod[l];
    }

    size_t P(uint32_t level) const { return (size_t)(level + 1) * n; }  // one polynomial

    Ct make(uint32_t level, double scale)
    {
        Ct r = std::make_shared<Batch>();
        r->c = c;
        r->level = level;
        r->scale = scale;
        if (!dry) {
            r->d = c->alloc((size_t)S * 2 * P(level));
            if (!r->d) PFAIL(HEC_ENOMEM, "ciphertext allocation");
        }
        return r;
    }

    void rescale(const Ct &ct)
    {
        if (ct->level == 0) PFAIL(HEC_ELEVEL, "cannot rescale at level 0");
        if (!dry) PTRY(rescale_polys(c, &ct->d, ct->level, (int)(2 * S)));
        ct->scale /= (double)c->mod[ct->level];
        ct->level -= 1;
    }

    ScalarArg scalar(double value, double scale, uint32_t nlimbs)
    {
        int64_t m;
        PTRY(const_coeff(value, scale, &m));
        ScalarArg sa;
        if (!dry) scalar_arg(c, m, nlimbs, sa);
        return sa;
    }

    // ct dropped to level l (l <= ct's level) times value at S[l-1] q_l / ct.scale, not rescaled; nominal
    // scale S[l-1] q_l
    Ct const_mul_raw(const Ct &ct, double value, uint32_t l)
    {
        if (l == 0) PFAIL(HEC_ELEVEL, "polynomial evaluation ran out of levels");
        if (l > ct->level) PFAIL(HEC_ELEVEL, "cannot raise a level");
        const double pscale = S_[l - 1] * (double)c->mod[l] / ct->scale;
        const ScalarArg sa = scalar(value, pscale, l + 1);
        Ct r = make(l, S_[l - 1] * (double)c->mod[l]);
        if (!dry)
            hec_scalar(c->T, SC_MUL, r->d, ct->d, P(l), P(ct->level), (int)(2 * S), (int)l + 1, 0, sa, c->st);
        return r;
    }

    // ct dropped to level l (default: its own) times value, rescaled to level l-1 at the nominal scale S[l-1]
    Ct const_mul(const Ct &ct, double value, uint32_t l = UINT32_MAX)
    {
        if (l == UINT32_MAX) l = ct->level;
        Ct r = const_mul_raw(ct, value, l);
        rescale(r);
        r->scale = S_[l - 1];
        return r;
    }

    // ct brought down to `level`: limbs dropped to level + 1, times 1 (cached per batch and level; the cache
    // keeps the source alive, so its address is not reused)
    std::map<std::pair<const Batch *, uint32_t>, std::pair<Ct, Ct>> adj;
    Ct adjust(const Ct &ct, uint32_t level)
    {
        if (ct->level == level) return ct;
        if (ct->level < level) PFAIL(HEC_ELEVEL, "cannot raise a level");
        auto key = std::make_pair((const Batch *)ct.get(), level);
        auto it = adj.find(key);
        if (it != adj.end()) return it->second.second;
        Ct r = const_mul(ct, 1.0, level + 1);
        adj[key] = std::make_pair(ct, r);
        return r;
    }

    // relinearized products of the S pairs: tensor product, ModUp of the s^2
    // parts, key switch with the relinearization key, ModDown, added to (d0, d1);
    // the pairs are the items' batches one after the other (S / items.size() each)
    Ct product(const std::vector<Ct> &us, const std::vector<Ct> &vs)
    {
        const Ct &u = us[0], &v = vs[0];
        const uint32_t l = u->level, nq = l + 1, nqp = nq + c->k;
        const uint32_t beta = (nq + c->alpha - 1) / c->alpha;
        Ct r = make(l, u->scale * v->scale);
        if (dry) return r;
        const u64 *rlk = nullptr;
        PTRY(relin_key(c, &rlk));
        const size_t p = P(l);
        // t_i = [d0][d2][d1]: a ciphertext view (d0, d2) whose second polynomial is the one ModUp reads
        u64 *t = c->alloc((size_t)S * 3 * p), *E = c->alloc((size_t)S * 2 * nqp * n);
        if (!t || !E) {
            c->release(t);
            c->release(E);
            PFAIL(HEC_ENOMEM, "ciphertext product buffers");
        }
        if (us.size() == 1) {
            hec_tensor(c->T, t, u->d, v->d, (int)nq, (int)S, c->st);
        } else {
            TensorItems ti{};
            for (size_t j = 0; j < us.size(); j++) {
                ti.a[j] = us[j]->d;
                ti.b[j] = vs[j]->d;
            }
            if (!hec_tensor_items(c->T, t, ti, (int)us.size(), (int)(S / us.size()), (int)nq, c->st)) {
                c->release(t);
                c->release(E);
                PFAIL(HEC_EINVAL, "invalid tensor batch");
            }
        }
        std::vector<hec_ct> tv(S), ov(S);
        std::vector<const hec_ct *> tp(S);
        std::vector<hec_ct *> op(S);
        for (uint32_t i = 0; i < S; i++) {
            tv[i].ctx = ov[i].ctx = c;
            tv[i].level = ov[i].level = l;
            tv[i].d = t + (size_t)i * 3 * p;
            ov[i].d = r->d + (size_t)i * 2 * p;
            tp[i] = &tv[i];
            op[i] = &ov[i];
        }
        u64 *D = nullptr;
        hec_status s = ct_modup_many(c, tp, &D);
        for (uint32_t b0 = 0; b0 < S && s == HEC_OK; b0 += HEC_KS_BATCH) {
            const uint32_t R = std::min((uint32_t)HEC_KS_BATCH, S - b0);
            KsBatch kb{};
            for (uint32_t q = 0; q < R; q++) {
                kb.key[q] = rlk;
                kb.out[q] = E + (size_t)(b0 + q) * 2 * nqp * n;
                kb.D[q] = D + (size_t)(b0 + q) * beta * nqp * n;
                kb.g[q] = 1;
            }
            hec_ks_inner(c->T, kb, (int)R, nullptr, (int)beta, (int)nqp, c->qpmap(l), (int)c->NLK, c->st);
        }
        c->ks_count += S;
        // ModDown of every key-switched d2 plus its (d0, d1), at t_i and t_i + 2p
        std::vector<std::array<const u64 *, 2>> adds(S);
        for (uint32_t i = 0; i < S; i++) adds[i] = {t + (size_t)i * 3 * p, t + (size_t)i * 3 * p + 2 * p};
        if (s == HEC_OK) s = ct_moddown_many(c, l, E, op, &adds);
        for (auto &h : tv) h.d = nullptr;
        for (auto &h : ov) h.d = nullptr;
        c->release(D);
        c->release(t);
        c->release(E);
        PTRY(s);
        return r;
    }

    Ct mul(const Ct &u0, const Ct &v0) { return muls({{u0, v0}})[0]; }

    // several independent rescaled products, each at the lower level of its
    // operands; those at one level go as one batch: the operands are gathered
    // side by side, multiplied, rescaled and split again
    std::vector<Ct> muls(const std::vector<std::pair<Ct, Ct>> &pairs)
    {
        std::vector<Ct> out(pairs.size());
        std::map<uint32_t, std::vector<size_t>> by_level;
        for (size_t i = 0; i < pairs.size(); i++)
            by_level[std::min(pairs[i].first->level, pairs[i].second->level)].push_back(i);
        for (auto &kv : by_level) {
            const uint32_t l = kv.first;
            const std::vector<size_t> &idx = kv.second;
            const size_t K = idx.size();
            if (l == 0) PFAIL(HEC_ELEVEL, "polynomial evaluation ran out of levels");
            std::vector<Ct> us, vs;
            for (size_t i : idx) {
                us.push_back(adjust(pairs[i].first, l));
                vs.push_back(adjust(pairs[i].second, l));
            }
            Ct r;
            if (K == 1) {
                r = product(us, vs);
                rescale(r);
            } else {
                // the operands read in place (items of the tensor launch) or, beyond
                // HEC_TENSOR_ITEMS of them, gathered side by side first
                std::vector<Ct> U = us, V = vs;
                if (K > HEC_TENSOR_ITEMS) {
                    U = {gather(us)};
                    V = {gather(vs)};
                }
                const uint32_t S0 = S;
                S = S0 * (uint32_t)K;
                try {
                    r = product(U, V);
                    rescale(r);
                } catch (...) {
                    S = S0;
                    throw;
                }
                S = S0;
            }
            if (r->scale != S_[l - 1]) PFAIL(HEC_ESCALE, "product scale off the scale table");
            std::vector<Ct> parts = K == 1 ? std::vector<Ct>{r} : split(r, K);
            for (size_t j = 0; j < K; j++) out[idx[j]] = parts[j];
        }
        return out;
    }

    // K batches at one level and scale side by side (and back)
    Ct gather(const std::vector<Ct> &xs)
    {
        const uint32_t S0 = S;
        S = S0 * (uint32_t)xs.size();
        Ct g;
        try {
            g = make(xs[0]->level, xs[0]->scale);
        } catch (...) {
            S = S0;
            throw;
        }
        S = S0;
        if (!dry) {
            const size_t bytes = (size_t)S * 2 * P(xs[0]->level) * 8;
            for (size_t i = 0; i < xs.size(); i++)
                if (hipMemcpyAsync((char *)g->d + i * bytes, xs[i]->d, bytes, hipMemcpyDeviceToDevice, c->st) !=
                    hipSuccess)
                    PFAIL(HEC_EDEVICE, "gather copy");
        }
        return g;
    }
    std::vector<Ct> split(const Ct &g, size_t K)
    {
        std::vector<Ct> out;
        const size_t bytes = (size_t)S * 2 * P(g->level) * 8;
        for (size_t i = 0; i < K; i++) {
            Ct r = make(g->level, g->scale);
            if (!dry && hipMemcpyAsync(r->d, (const char *)g->d + i * bytes, bytes, hipMemcpyDeviceToDevice, c->st) !=
                            hipSuccess)
                PFAIL(HEC_EDEVICE, "split copy");
            out.push_back(r);
        }
        return out;
    }

    Ct ew(EwOp op, const Ct &u, const Ct &v)
    {
        if (u->level != v->level || u->scale != v->scale) PFAIL(HEC_ESCALE, "level/scale mismatch");
        Ct r = make(u->level, u->scale);
        if (!dry) {
            const size_t p = P(u->level);
            hec_ew(c->T, op, r->d, u->d, v->d, p, p, p, (int)(2 * S), c->idmap(), (int)u->level + 1, c->st);
        }
        return r;
    }

    Ct add(const Ct &u, const Ct &v)
    {
        const uint32_t l = std::min(u->level, v->level);
        return ew(EW_ADD, adjust(u, l), adjust(v, l));
    }

    // u + v, or 2u + v with dbl (v encoded at u's scale)
    Ct add_const(const Ct &u, double v, bool dbl = false)
    {
        const ScalarArg sa = scalar(v, u->scale, u->level + 1);
        Ct r = make(u->level, u->scale);
        if (!dry) {
            const size_t p = P(u->level);
            hec_scalar(c->T, dbl ? SC_DBL_ADD : SC_ADD, r->d, u->d, p, p, (int)(2 * S), (int)u->level + 1, 0, sa,
                       c->st);
        }
        return r;
    }

    // y = alpha x + beta maps [a, b] onto [-1, 1]; on [-1, 1] itself y = x (no level spent)
    Ct affine()
    {
        if (a == -1.0 && b == 1.0) return x;
        const double alpha = 2.0 / (b - a);
        const double beta = -(a + b) / (b - a);
        return add_const(const_mul(x, alpha), beta);
    }

    // T_k for 2 <= k < min(m, d + 1) and the giant powers T_m, T_2m, ... <= d.  The
    // products of one doubling round (T_k for 2^i < k <= 2^(i+1), all from
    // T_1..T_(2^i)) are independent and taken as one batch; the giant powers
    // of the same round join it.
    void basis(const Ct &y, uint32_t m, uint32_t d, std::map<uint32_t, Ct> &T)
    {
        T[1] = y;
        const uint32_t top = std::min(m, d + 1);  // babies are T_k, k < top
        for (uint32_t lo = 1; lo < std::max(top - 1, m); lo *= 2) {
            std::vector<uint32_t> ks;
            for (uint32_t k = lo + 1; k <= 2 * lo; k++)
                if (k < top || (k == m && m <= d)) ks.push_back(k);
            if (ks.empty()) break;
            std::vector<std::pair<Ct, Ct>> pairs;
            for (uint32_t k : ks)
                pairs.push_back(k % 2 == 0 ? std::make_pair(T[k / 2], T[k / 2]) : std::make_pair(T[k / 2 + 1], T[k / 2]));
            std::vector<Ct> ps = muls(pairs);
            for (size_t i = 0; i < ks.size(); i++) {
                const uint32_t k = ks[i];
                if (k % 2 == 0) T[k] = add_const(ps[i], -1.0, true);  // 2 T_{k/2}^2 - 1
                else T[k] = ew(EW_DBL_SUB, ps[i], adjust(T[1], ps[i]->level));  // 2 T_{h+1} T_h - T_1
            }
        }
        for (uint32_t g = 2 * m; g <= d; g *= 2) {
            Ct p = mul(T[g / 2], T[g / 2]);
            T[g] = add_const(p, -1.0, true);
        }
        if (m <= d && !T.count(m)) {
            Ct p = mul(T[m / 2], T[m / 2]);
            T[m] = add_const(p, -1.0, true);
        }
    }

    Val lin(const std::vector<double> &cf, std::map<uint32_t, Ct> &T)
    {
        std::vector<uint32_t> js;
        for (uint32_t j = 1; j < cf.size(); j++)
            if (cf[j] != 0.0) js.push_back(j);
        if (js.empty()) return Val::constant(cf[0]);
        uint32_t lo = UINT32_MAX;
        for (uint32_t j : js) lo = std::min(lo, T[j]->level);
        if (lo == 0) PFAIL(HEC_ELEVEL, "polynomial evaluation ran out of levels");
        const uint32_t top = lo - 1, l = top + 1;
        // every T_j dropped to top + 1 and multiplied by c_j, summed in one pass (one launch for up to
        // HEC_LIN_TERMS terms), the sum rescaled once
        Ct acc = make(l, S_[l - 1] * (double)c->mod[l]);
        const bool fused = js.size() <= HEC_LIN_TERMS && l + 1 <= HEC_LIN_LIMBS;
        LinArg la{};
        bool first = true;
        for (size_t i = 0; i < js.size(); i++) {
            const uint32_t j = js[i];
            const double pscale = S_[l - 1] * (double)c->mod[l] / T[j]->scale;
            const ScalarArg sa = scalar(cf[j], pscale, l + 1);
            if (dry) continue;
            if (fused) {
                la.in[i] = T[j]->d;
                la.ps[i] = P(T[j]->level);
                for (uint32_t r = 0; r <= l; r++) la.cm[i][r] = (u64)(((hec::u128)sa.v[r] << 64) % c->mod[r]);
            } else {
                hec_scalar(c->T, SC_MAC, acc->d, T[j]->d, P(l), P(T[j]->level), (int)(2 * S), (int)l + 1,
                           first ? 1 : 0, sa, c->st);
            }
            first = false;
        }
        if (!dry && fused && !hec_lincomb(c->T, acc->d, P(l), (int)(2 * S), (int)l + 1, la, (int)js.size(), c->st))
            PFAIL(HEC_EINVAL, "invalid linear-combination launch");
        rescale(acc);
        acc->scale = S_[top];
        return Val::of(cf[0] != 0.0 ? add_const(acc, cf[0]) : acc);
    }

    Val sum(Val u, Val v)
    {
        if (u.is_const && v.is_const) return Val::constant(u.c + v.c);
        if (u.is_const) std::swap(u, v);
        if (v.is_const) return v.c != 0.0 ? Val::of(add_const(u.ct, v.c)) : u;
        return Val::of(add(u.ct, v.ct));
    }

    // The division tree of the polynomial: leaves are the baby-step
    // combinations (evaluated as the tree is built, they need no product),
    // inner nodes q T_g + r.  The products q T_g are then taken in rounds by
    // their depth in the tree, those of one round (and one level) as one batch;
    // every value is the one the depth-first order gives.
    struct Node {
        int kind = 0;  // 0 value, 1 product Q * T_g, 2 sum
        Val v;
        bool done = false;
        int a = -1, b = -1;  // product: Q node; sum: P and R nodes
        uint32_t g = 0, height = 0;
    };
    std::vector<Node> nodes;

    int leaf(Val v)
    {
        Node nd;
        nd.v = std::move(v);
        nd.done = true;
        nodes.push_back(nd);
        return (int)nodes.size() - 1;
    }

    int build(const std::vector<double> &cf, std::map<uint32_t, Ct> &T, uint32_t m)
    {
        const uint32_t d = (uint32_t)cf.size() - 1;
        if (d < m) return leaf(lin(cf, T));
        uint32_t g = m;
        while (2 * g <= d) g *= 2;
        std::vector<double> q, r;
        cheb_divide(cf, g, q, r);
        const int Q = build(q, T, m);
        int P;
        if (nodes[Q].kind == 0 && nodes[Q].v.is_const) {
            const double qc = nodes[Q].v.c;
            P = leaf(qc != 0.0 ? Val::of(const_mul(T[g], qc)) : Val::constant(0.0));
        } else {
            Node nd;
            nd.kind = 1;
            nd.a = Q;
            nd.g = g;
            nd.height = nodes[Q].height + 1;
            nodes.push_back(nd);
            P = (int)nodes.size() - 1;
        }
        const int R = build(r, T, m);
        Node nd;
        nd.kind = 2;
        nd.a = P;
        nd.b = R;
        nd.height = std::max(nodes[P].height, nodes[R].height);
        nodes.push_back(nd);
        return (int)nodes.size() - 1;
    }

    // the value of a node whose products are all taken
    Val value(int i)
    {
        Node &nd = nodes[i];
        if (nd.done) return nd.v;
        if (nd.kind != 2) PFAIL(HEC_EINVAL, "product evaluated out of order");
        Val pv = value(nd.a), rv = value(nd.b);
        nodes[i].v = sum(pv, rv);
        nodes[i].done = true;
        return nodes[i].v;
    }

    Val ev(const std::vector<double> &cf, std::map<uint32_t, Ct> &T, uint32_t m)
    {
        nodes.clear();
        const int root = build(cf, T, m);
        uint32_t H = 0;
        for (auto &nd : nodes)
            if (nd.kind == 1) H = std::max(H, nd.height);
        for (uint32_t h = 1; h <= H; h++) {
            std::vector<int> ids;
            std::vector<std::pair<Ct, Ct>> pairs;
            for (int i = 0; i < (int)nodes.size(); i++)
                if (nodes[i].kind == 1 && nodes[i].height == h) {
                    Val q = value(nodes[i].a);
                    if (q.is_const) {  // a quotient that summed to a constant: a constant product
                        nodes[i].v = q.c != 0.0 ? Val::of(const_mul(T[nodes[i].g], q.c)) : Val::constant(0.0);
                        nodes[i].done = true;
                        continue;
                    }
                    ids.push_back(i);
                    pairs.push_back({q.ct, T[nodes[i].g]});
                }
            if (ids.empty()) continue;
            std::vector<Ct> ps = muls(pairs);
            for (size_t j = 0; j < ids.size(); j++) {
                nodes[ids[j]].v = Val::of(ps[j]);
                nodes[ids[j]].done = true;
            }
        }
        return value(root);
    }

    // p = q T_g + r for g <= deg p < 2g; ascending j, each step one IEEE operation
    static void cheb_divide(const std::vector<double> &cf, uint32_t g, std::vector<double> &q, std::vector<double> &r)
    {
        const uint32_t d = (uint32_t)cf.size() - 1;
        q.assign(d - g + 1, 0.0);
        r.assign(cf.begin(), cf.begin() + g);
        q[0] = cf[g];
        for (uint32_t j = g + 1; j <= d; j++) {
            q[j - g] = 2.0 * cf[j];
            r[2 * g - j] = r[2 * g - j] - cf[j];
        }
    }

    static uint32_t baby_size(uint32_t d)
    {
        uint32_t m = 1;
        while ((uint64_t)m * m < (uint64_t)d + 1) m *= 2;
        return m;
    }

    Ct run(const std::vector<double> &cf)
    {
        const uint32_t d = (uint32_t)cf.size() - 1;
        const uint32_t m = baby_size(d);
        std::map<uint32_t, Ct> T;
        basis(affine(), m, d, T);
        Val r = ev(cf, T, m);
        if (r.is_const) PFAIL(HEC_EINVAL, "the polynomial is constant");
        return r.ct;
    }
};

hec_status check_args(hec_ctx *c, const double *coeffs, size_t n, double a, double b)
{
    if (!c->have_keys) HEC_FAIL(HEC_ENOKEY, "ckks_keygen has not been called");
    if (!coeffs || n < 2) HEC_FAIL(HEC_EINVAL, "need at least two coefficients (degree >= 1)");
    if (n > 4096) HEC_FAIL(HEC_EINVAL, "degree above 4095");
    for (size_t i = 0; i < n; i++)
        if (!std::isfinite(coeffs[i])) HEC_FAIL(HEC_EINVAL, "coefficient %zu not finite", i);
    if (!std::isfinite(a) || !std::isfinite(b) || !(b > a)) HEC_FAIL(HEC_EINVAL, "interval must satisfy a < b");
    return HEC_OK;
}

// levels and scales only: output level and scale of an input (level, scale)
hec_status cheb_dry(hec_ctx *c, uint32_t level, double scale, const std::vector<double> &cf, double a, double b,
                    uint32_t *out_level, double *out_scale)
{
    try {
        Ct x = std::make_shared<Batch>();
        x->level = level;
        x->scale = scale;
        ChebEval ev(c, x, 1, a, b, true);
        Ct r = ev.run(cf);
        *out_level = r->level;
        if (out_scale) *out_scale = r->scale;
        return HEC_OK;
    } catch (const Fail &f) {
        return f.s;
    } catch (const std::bad_alloc &) {
        HEC_FAIL(HEC_ENOMEM, "host allocation");
    }
}

}  // namespace

hec_status cheb_levels(hec_ctx *c, uint32_t level, double scale, const double *coeffs, size_t n, double a, double b,
                       uint32_t *out_level, double *out_scale)
{
    HEC_CHECK(check_args(c, coeffs, n, a, b));
    return cheb_dry(c, level, scale, std::vector<double>(coeffs, coeffs + n), a, b, out_level, out_scale);
}

hec_status cheb_image(hec_ctx *c, const std::vector<hec_ct *> &in, const double *coeffs, size_t n, double a, double b,
                      std::vector<hec_ct *> &out)
{
    out.clear();
    HEC_CHECK(check_args(c, coeffs, n, a, b));
    if (in.empty()) HEC_FAIL(HEC_ELAYOUT, "nothing to evaluate");
    const uint32_t lvl = in[0]->level;
    const double scale = in[0]->scale;
    for (auto *x : in)
        if (x->level != lvl || x->scale != scale) HEC_FAIL(HEC_ELEVEL, "ciphertexts at different levels or scales");
    std::vector<double> cf(coeffs, coeffs + n);
    uint32_t olvl = 0;
    HEC_CHECK(cheb_dry(c, lvl, scale, cf, a, b, &olvl, nullptr));  // levels and constants before any launch
    const uint32_t S = (uint32_t)in.size();
    const size_t pc = (size_t)2 * (lvl + 1) * c->n;
    hec_status s = HEC_OK;
    try {
        // the shards side by side, evaluated together, then handed out one by one
        Ct x = std::make_shared<Batch>();
        x->c = c;
        x->level = lvl;
        x->scale = scale;
        x->d = c->alloc((size_t)S * pc);
        if (!x->d) PFAIL(HEC_ENOMEM, "ciphertext allocation");
        for (uint32_t i = 0; i < S; i++)
            if (hipMemcpyAsync(x->d + i * pc, in[i]->d, pc * 8, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
                PFAIL(HEC_EDEVICE, "shard copy");
        ChebEval ev(c, x, S, a, b, false);
        Ct r = ev.run(cf);
        const size_t po = (size_t)2 * (r->level + 1) * c->n;
        for (uint32_t i = 0; i < S; i++) {
            hec_ct *o = ct_new(c, r->level, r->scale);
            if (!o) PFAIL(HEC_ENOMEM, "ciphertext allocation");
            out.push_back(o);
            if (hipMemcpyAsync(o->d, r->d + i * po, po * 8, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
                PFAIL(HEC_EDEVICE, "result copy");
        }
    } catch (const Fail &f) {
        s = f.s;
    } catch (const std::bad_alloc &) {
        s = HEC_ENOMEM;
        hec_set_error("host allocation");
    }
    if (s == HEC_OK && hipGetLastError() != hipSuccess) {
        s = HEC_EDEVICE;
        hec_set_error("kernel launch failed");
    }
    if (s != HEC_OK) {
        for (auto *p : out) ct_free(p);
        out.clear();
    }
    return s;
}

extern "C" hec_status he_cheb_eval(hec_ctx *c, const hec_ct *x, const double *coeffs, size_t ncoeffs, double a,
                                   double b, hec_ct **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !x) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    std::vector<hec_ct *> o;
    HEC_CHECK(cheb_image(c, {const_cast<hec_ct *>(x)}, coeffs, ncoeffs, a, b, o));
    *out = o[0];
    return HEC_OK;
}

extern "C" hec_status he_image_cheb_eval(hec_ctx *c, const hec_image *in, const double *coeffs, size_t ncoeffs,
                                         double a, double b, hec_image **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !in) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (in->shards.empty()) HEC_FAIL(HEC_ELAYOUT, "empty image");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    hec_image *im = new hec_image();
    im->ctx = c;
    im->lay = in->lay;
    hec_status s = cheb_image(c, in->shards, coeffs, ncoeffs, a, b, im->shards);
    if (s != HEC_OK) {
        hec_image_free(im);
        return s;
    }
    *out = im;
    return HEC_OK;
}
