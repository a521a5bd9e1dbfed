// hec_poly.cpp -- polynomial evaluation on ciphertexts in the Chebyshev basis
// (the activation of the encrypted network, Sec. II-C: a polynomial
// approximation over a fixed interval evaluated with ciphertext products),
// with baby-step/giant-step splitting of the polynomial.
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
// sum rescaled once; a larger one is divided by the
// largest giant power T_g <= its degree (T_j = 2 T_g T_{j-g} - T_{2g-j}),
// p = q T_g + r, and q, r are evaluated the same way.
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

using Ct = std::shared_ptr<hec_ct>;
Ct wrap(hec_ct *p) { return Ct(p, ct_free); }

// a ciphertext or a plain constant (sums of constants stay on the host)
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

// dry: levels and scales only (ciphertexts without device data), to learn the
// output level and check the level budget and constants before any launch
struct ChebEval {
    hec_ctx *c;
    Ct x;
    double a, b;
    bool dry;
    std::vector<double> S;  // nominal scale per level

    ChebEval(hec_ctx *ctx, Ct in, double lo, double hi, bool dry_run = false)
        : c(ctx), x(std::move(in)), a(lo), b(hi), dry(dry_run)
    {
        S.assign(x->level + 1, 0.0);
        S[x->level] = x->scale;
        for (uint32_t l = x->level; l > 0; l--) S[l - 1] = (S[l] * S[l]) / (double)c->mod[l];
    }

    Ct meta(uint32_t level, double scale)
    {
        hec_ct *o = new hec_ct();
        o->ctx = c;
        o->level = level;
        o->scale = scale;
        return wrap(o);
    }

    void rescale(const Ct &ct)
    {
        if (!dry) {
            PTRY(ct_rescale(c, ct.get()));
            return;
        }
        if (ct->level == 0) PFAIL(HEC_ELEVEL, "cannot rescale at level 0");
        ct->scale /= (double)c->mod[ct->level];
        ct->level -= 1;
    }

    // ct dropped to level l (l <= ct's level) times value at S[l-1] q_l / ct.scale, not rescaled; nominal
    // scale S[l-1] q_l
    Ct const_mul_raw(const Ct &ct, double value, uint32_t l)
    {
        if (l == 0) PFAIL(HEC_ELEVEL, "polynomial evaluation ran out of levels");
        if (l > ct->level) PFAIL(HEC_ELEVEL, "cannot raise a level");
        const double pscale = S[l - 1] * (double)c->mod[l] / ct->scale;
        Ct r;
        if (dry) {
            int64_t m;
            PTRY(const_coeff(value, pscale, &m));
            r = meta(l, 0.0);
        } else {
            hec_ct *o = nullptr;
            PTRY(ct_mul_const_at(c, ct.get(), l, value, pscale, &o));
            r = wrap(o);
        }
        r->scale = S[l - 1] * (double)c->mod[l];
        return r;
    }

    // ct dropped to level l (default: its own) times value, rescaled to level l-1 at the nominal scale S[l-1]
    Ct const_mul(const Ct &ct, double value, uint32_t l = UINT32_MAX)
    {
        if (l == UINT32_MAX) l = ct->level;
        Ct r = const_mul_raw(ct, value, l);
        rescale(r);
        r->scale = S[l - 1];
        return r;
    }

    // ct brought down to `level`: limbs dropped to level + 1, times 1 (cached per ciphertext and level; the
    // cache keeps the source alive, so its address is not reused)
    std::map<std::pair<const hec_ct *, uint32_t>, std::pair<Ct, Ct>> adj;
    Ct adjust(const Ct &ct, uint32_t level)
    {
        if (ct->level == level) return ct;
        if (ct->level < level) PFAIL(HEC_ELEVEL, "cannot raise a level");
        auto key = std::make_pair((const hec_ct *)ct.get(), level);
        auto it = adj.find(key);
        if (it != adj.end()) return it->second.second;
        Ct r = const_mul(ct, 1.0, level + 1);
        adj[key] = std::make_pair(ct, r);
        return r;
    }

    Ct mul(const Ct &u0, const Ct &v0)
    {
        const uint32_t l = std::min(u0->level, v0->level);
        if (l == 0) PFAIL(HEC_ELEVEL, "polynomial evaluation ran out of levels");
        Ct u = adjust(u0, l), v = adjust(v0, l);
        Ct r;
        if (dry) {
            r = meta(l, u->scale * v->scale);
        } else {
            hec_ct *o = nullptr;
            PTRY(ct_mul(c, u.get(), v.get(), &o));
            r = wrap(o);
        }
        rescale(r);
        if (r->scale != S[l - 1]) PFAIL(HEC_ESCALE, "product scale off the scale table");
        return r;
    }

    Ct add_raw(const Ct &u, const Ct &v)
    {
        if (u->level != v->level || u->scale != v->scale) PFAIL(HEC_ESCALE, "level/scale mismatch in addition");
        if (dry) return meta(u->level, u->scale);
        hec_ct *o = nullptr;
        PTRY(ct_add(c, u.get(), v.get(), &o));
        return wrap(o);
    }

    Ct add(const Ct &u, const Ct &v)
    {
        const uint32_t l = std::min(u->level, v->level);
        return add_raw(adjust(u, l), adjust(v, l));
    }

    Ct add_const(const Ct &u, double v)
    {
        if (dry) {
            int64_t m;
            PTRY(const_coeff(v, u->scale, &m));
            return meta(u->level, u->scale);
        }
        hec_ct *o = nullptr;
        PTRY(ct_add_const(c, u.get(), v, u->scale, &o));
        return wrap(o);
    }

    // 2u + v (v at u's scale)
    Ct dbl_add_const(const Ct &u, double v)
    {
        if (dry) {
            int64_t m;
            PTRY(const_coeff(v, u->scale, &m));
            return meta(u->level, u->scale);
        }
        hec_ct *o = nullptr;
        PTRY(ct_dbl_add_const(c, u.get(), v, &o));
        return wrap(o);
    }

    // 2u - v
    Ct dbl_sub(const Ct &u, const Ct &v)
    {
        if (dry) {
            if (u->level != v->level || u->scale != v->scale) PFAIL(HEC_ESCALE, "level/scale mismatch");
            return meta(u->level, u->scale);
        }
        hec_ct *o = nullptr;
        PTRY(ct_dbl_sub(c, u.get(), v.get(), &o));
        return wrap(o);
    }

    Ct sub(const Ct &u, const Ct &v)
    {
        if (dry) {
            if (u->level != v->level || u->scale != v->scale) PFAIL(HEC_ESCALE, "level/scale mismatch");
            return meta(u->level, u->scale);
        }
        hec_ct *o = nullptr;
        PTRY(ct_sub(c, u.get(), v.get(), &o));
        return wrap(o);
    }

    // y = alpha x + beta maps [a, b] onto [-1, 1]; on [-1, 1] itself y = x (no level spent)
    Ct affine()
    {
        if (a == -1.0 && b == 1.0) return x;
        const double alpha = 2.0 / (b - a);
        const double beta = -(a + b) / (b - a);
        return add_const(const_mul(x, alpha), beta);
    }

    void basis(const Ct &y, uint32_t m, uint32_t d, std::map<uint32_t, Ct> &T)
    {
        T[1] = y;
        for (uint32_t k = 2; k < std::min(m, d + 1); k++) {
            if (k % 2 == 0) {
                Ct p = mul(T[k / 2], T[k / 2]);
                T[k] = dbl_add_const(p, -1.0);
            } else {
                const uint32_t h = k / 2;
                Ct p = mul(T[h + 1], T[h]);
                T[k] = dbl_sub(p, adjust(T[1], p->level));
            }
        }
        for (uint32_t g = m; g <= d; g *= 2) {
            Ct p = mul(T[g / 2], T[g / 2]);
            T[g] = dbl_add_const(p, -1.0);
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
        const uint32_t top = lo - 1;
        // every T_j dropped to top + 1 and multiplied by c_j, accumulated in one buffer, the sum rescaled once
        const uint32_t l = top + 1;
        Ct acc;
        if (dry) {
            for (uint32_t j : js) const_mul_raw(T[j], cf[j], l);
            acc = meta(l, 0.0);
        } else {
            hec_ct *o = ct_new(c, l, 1.0);
            if (!o) PFAIL(HEC_ENOMEM, "ciphertext allocation");
            acc = wrap(o);
            bool first = true;
            for (uint32_t j : js) {
                const double pscale = S[l - 1] * (double)c->mod[l] / T[j]->scale;
                PTRY(ct_mac_const(c, acc.get(), T[j].get(), cf[j], pscale, first));
                first = false;
            }
        }
        acc->scale = S[l - 1] * (double)c->mod[l];
        rescale(acc);
        acc->scale = S[top];
        return Val::of(cf[0] != 0.0 ? add_const(acc, cf[0]) : acc);
    }

    Val sum(Val u, Val v)
    {
        if (u.is_const && v.is_const) return Val::constant(u.c + v.c);
        if (u.is_const) std::swap(u, v);
        if (v.is_const) return v.c != 0.0 ? Val::of(add_const(u.ct, v.c)) : u;
        return Val::of(add(u.ct, v.ct));
    }

    Val ev(const std::vector<double> &cf, std::map<uint32_t, Ct> &T, uint32_t m)
    {
        const uint32_t d = (uint32_t)cf.size() - 1;
        if (d < m) return lin(cf, T);
        uint32_t g = m;
        while (2 * g <= d) g *= 2;
        std::vector<double> q, r;
        cheb_divide(cf, g, q, r);
        Val Q = ev(q, T, m);
        Val P;
        if (Q.is_const) P = Q.c != 0.0 ? Val::of(const_mul(T[g], Q.c)) : Val::constant(0.0);
        else P = Val::of(mul(Q.ct, T[g]));
        Val R = ev(r, T, m);
        return sum(P, R);
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

// the evaluation of one ciphertext (x borrowed), or with dry its level and scale only
hec_status cheb_one(hec_ctx *c, const hec_ct *x, const std::vector<double> &cf, double a, double b, bool dry,
                    hec_ct **out)
{
    try {
        hec_ct *xc = nullptr;
        if (dry) {
            xc = new hec_ct();
            xc->ctx = c;
            xc->level = x->level;
            xc->scale = x->scale;
        } else {
            xc = ct_clone(x);
            if (!xc) HEC_FAIL(HEC_ENOMEM, "ciphertext allocation");
        }
        ChebEval ev(c, wrap(xc), a, b, dry);
        Ct r = ev.run(cf);
        // move the result's storage into a handle of its own
        hec_ct *o = new hec_ct(*r);
        r->d = nullptr;
        *out = o;
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
    hec_ct x;
    x.ctx = c;
    x.level = level;
    x.scale = scale;
    hec_ct *r = nullptr;
    HEC_CHECK(cheb_one(c, &x, std::vector<double>(coeffs, coeffs + n), a, b, true, &r));
    *out_level = r->level;
    if (out_scale) *out_scale = r->scale;
    delete r;
    return HEC_OK;
}

hec_status cheb_image(hec_ctx *c, const std::vector<hec_ct *> &in, const double *coeffs, size_t n, double a, double b,
                      std::vector<hec_ct *> &out)
{
    HEC_CHECK(check_args(c, coeffs, n, a, b));
    std::vector<double> cf(coeffs, coeffs + n);
    out.clear();
    for (const hec_ct *x : in) {
        hec_ct *o = nullptr;
        hec_status s = cheb_one(c, x, cf, a, b, true, &o);  // levels and constants first
        delete o;
        o = nullptr;
        if (s == HEC_OK) s = cheb_one(c, x, cf, a, b, false, &o);
        if (s != HEC_OK) {
            for (auto *p : out) ct_free(p);
            out.clear();
            return s;
        }
        out.push_back(o);
    }
    if (hipGetLastError() != hipSuccess) {
        for (auto *p : out) ct_free(p);
        out.clear();
        HEC_FAIL(HEC_EDEVICE, "kernel launch failed");
    }
    return HEC_OK;
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
