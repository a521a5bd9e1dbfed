// hec_host.cpp -- host-side number theory, tables and the slot encoder.
#include "hec_host.h"

#include <cmath>
#include <complex>
#include <cstring>

namespace hec {

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

uint64_t powmod(uint64_t a, uint64_t e, uint64_t q)
{
    uint64_t r = 1 % q, x = a % q;
    for (; e; e >>= 1) {
        if (e & 1) r = mulmod(r, x, q);
        x = mulmod(x, x, q);
    }
    return r;
}

uint64_t invmod(uint64_t a, uint64_t q)
{
    // extended Euclid
    __int128 t = 0, nt = 1, r = q, nr = a % q;
    while (nr) {
        __int128 qq = r / nr, tmp;
        tmp = t - qq * nt; t = nt; nt = tmp;
        tmp = r - qq * nr; r = nr; nr = tmp;
    }
    if (t < 0) t += q;
    return (uint64_t)t;
}

// Miller-Rabin with a base set that is deterministic below 2^64
bool is_prime(uint64_t m)
{
    if (m < 2) return false;
    for (uint64_t p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull}) {
        if (m == p) return true;
        if (m % p == 0) return false;
    }
    uint64_t d = m - 1;
    int s = 0;
    while (!(d & 1)) { d >>= 1; s++; }
    for (uint64_t a : {2ull, 325ull, 9375ull, 28178ull, 450775ull, 9780504ull, 1795265022ull}) {
        a %= m;
        if (!a) continue;
        uint64_t x = powmod(a, d, m);
        if (x == 1 || x == m - 1) continue;
        bool comp = true;
        for (int i = 1; i < s && comp; i++) {
            x = mulmod(x, x, m);
            if (x == m - 1) comp = false;
        }
        if (comp) return false;
    }
    return true;
}

uint64_t find_prime(uint32_t bits, uint32_t n, const std::vector<uint64_t> &taken)
{
    const uint64_t top = 1ull << bits, step = 2ull * n, floor_ = 1ull << (bits - 1);
    for (uint64_t c = top - step + 1; c >= floor_ && c < top; c -= step) {
        if (!is_prime(c)) continue;
        bool used = false;
        for (uint64_t t : taken) used |= (t == c);
        if (!used) return c;
    }
    return 0;
}

uint64_t find_root_2n(uint64_t q, uint32_t n)
{
    for (uint64_t x = 2;; x++) {
        uint64_t g = powmod(x, (q - 1) / (2ull * n), q);
        if (powmod(g, n, q) == q - 1) return g;
    }
}

uint64_t shoup_of(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

void gauss_table(double sigma, uint64_t T[19])
{
    long double w[20], tot = 0;
    for (int i = 0; i <= 19; i++) {
        w[i] = (i ? 2.0L : 1.0L) * expl(-(long double)(i * i) / (2.0L * sigma * sigma));
        tot += w[i];
    }
    long double acc = 0;
    for (int i = 0; i < 19; i++) {
        acc += w[i];
        T[i] = (uint64_t)floorl(acc / tot * 9223372036854775808.0L);
    }
}

// ---------------------------------------------------------------------------
// double-double arithmetic (Dekker / Knuth error-free transformations)
// ---------------------------------------------------------------------------
namespace {
struct dd {
    double h, l;
};
inline dd two_sum(double a, double b)
{
    double s = a + b, bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
inline dd quick(double a, double b)
{
    double s = a + b;
    return {s, b - (s - a)};
}
inline dd two_prod(double a, double b)
{
    double p = a * b;
    return {p, std::fma(a, b, -p)};
}
inline dd add(dd x, dd y)
{
    dd s = two_sum(x.h, y.h), t = two_sum(x.l, y.l);
    s.l += t.h;
    s = quick(s.h, s.l);
    s.l += t.l;
    return quick(s.h, s.l);
}
inline dd neg(dd x) { return {-x.h, -x.l}; }
inline dd sub(dd x, dd y) { return add(x, neg(y)); }
inline dd mul(dd x, dd y)
{
    dd p = two_prod(x.h, y.h);
    p.l += x.h * y.l + x.l * y.h;
    return quick(p.h, p.l);
}
inline dd mul_d(dd x, double d)
{
    dd p = two_prod(x.h, d);
    p.l += x.l * d;
    return quick(p.h, p.l);
}
inline dd div_d(dd a, double b)
{
    double q1 = a.h / b;
    dd r = sub(a, two_prod(q1, b));
    double q2 = r.h / b;
    r = sub(r, two_prod(q2, b));
    double q3 = r.h / b;
    dd q = quick(q1, q2);
    return add(q, dd{q3, 0.0});
}
const dd PI = {3.141592653589793116, 1.2246467991473532e-16};

// cos and sin of x in [0, pi/4] by Taylor series in double-double
void sincos_dd(dd x, dd &c, dd &s)
{
    dd x2 = mul(x, x);
    dd term = x, sum = x;
    for (int k = 1; k < 30; k++) {
        term = div_d(mul(term, x2), (double)((2 * k) * (2 * k + 1)));
        sum = (k & 1) ? sub(sum, term) : add(sum, term);
        if (std::fabs(term.h) < 1e-36) break;
    }
    s = sum;
    term = {1.0, 0.0};
    sum = term;
    for (int k = 1; k < 30; k++) {
        term = div_d(mul(term, x2), (double)((2 * k - 1) * (2 * k)));
        sum = (k & 1) ? sub(sum, term) : add(sum, term);
        if (std::fabs(term.h) < 1e-36) break;
    }
    c = sum;
}

// round half away from zero of a double-double; |x| < 2^62 assumed
int64_t round_away(dd x, bool &ok)
{
    if (!(std::fabs(x.h) < 4611686018427387904.0)) { ok = false; return 0; }
    double f = std::floor(x.h);
    // frac = (x.h - f) + x.l ; x.h - f is exact for |x.h| < 2^52, and zero above
    double frac = (x.h - f) + x.l;
    int64_t base = (int64_t)f;
    // frac may have left [0, 1) through x.l
    while (frac >= 1.0) { frac -= 1.0; base += 1; }
    while (frac < 0.0) { frac += 1.0; base -= 1; }
    if (frac > 0.5) return base + 1;
    if (frac < 0.5) return base;
    // exact tie: away from zero
    return (base >= 0) ? base + 1 : base;
}
}  // namespace

Encoder::Encoder(uint32_t logn) : n_(1u << logn)
{
    const uint32_t n = n_, twon = 2 * n;
    ch_.resize(twon); cl_.resize(twon); sh_.resize(twon); sl_.resize(twon);
    const uint32_t quarter = n / 2;  // pi/2 in units of pi/n
    for (uint32_t e = 0; e < twon; e++) {
        uint32_t qd = e / quarter, r = e % quarter;
        bool flip = 2 * r > quarter;  // use pi/2 - phi
        uint32_t j = flip ? quarter - r : r;
        dd x = mul_d(PI, (double)j);
        x = {x.h / n, x.l / n};  // exact: n is a power of two
        dd c, s;
        sincos_dd(x, c, s);
        if (flip) std::swap(c, s);
        dd C, S;
        switch (qd & 3) {
        case 0: C = c; S = s; break;
        case 1: C = neg(s); S = c; break;
        case 2: C = neg(c); S = neg(s); break;
        default: C = s; S = neg(c); break;
        }
        ch_[e] = C.h; cl_[e] = C.l; sh_[e] = S.h; sl_[e] = S.l;
    }
    slot_root_.resize(n / 2);
    uint64_t f = 1;
    for (uint32_t j = 0; j < n / 2; j++) {
        slot_root_[j] = (uint32_t)((f - 1) / 2);
        f = f * 5 % twon;
    }
}

bool Encoder::encode(const double *z, size_t nz, double scale, int64_t *m) const
{
    const uint32_t n = n_, twon = 2 * n;
    std::vector<dd> re(n, dd{0, 0}), im(n, dd{0, 0});
    for (uint32_t j = 0; j < n / 2 && j < nz; j++) {
        uint32_t k = slot_root_[j];
        re[k] = dd{z[j], 0};            // root zeta^(5^j)
        re[n - 1 - k] = dd{z[j], 0};    // root zeta^(-5^j): (2n - f - 1)/2 = n - 1 - (f-1)/2
    }
    // bit reversal
    for (uint32_t i = 1, j = 0; i < n; i++) {
        uint32_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { std::swap(re[i], re[j]); std::swap(im[i], im[j]); }
    }
    // X[t] = sum_k v_k exp(-2 pi i k t / n)
    for (uint32_t len = 2; len <= n; len <<= 1) {
        uint32_t h = len / 2, step = 2 * (n / len);  // exp(-2 pi i j/len) = angle index 2j(n/len)
        for (uint32_t i = 0; i < n; i += len)
            for (uint32_t j = 0; j < h; j++) {
                uint32_t e = j * step;
                dd wr = {ch_[e], cl_[e]}, wi = {-sh_[e], -sl_[e]};
                dd br = re[i + j + h], bi = im[i + j + h];
                dd vr, vi;
                if (j == 0) { vr = br; vi = bi; }
                else {
                    vr = sub(mul(br, wr), mul(bi, wi));
                    vi = add(mul(br, wi), mul(bi, wr));
                }
                dd ar = re[i + j], ai = im[i + j];
                re[i + j] = add(ar, vr); im[i + j] = add(ai, vi);
                re[i + j + h] = sub(ar, vr); im[i + j + h] = sub(ai, vi);
            }
    }
    const double sc = scale / (double)n;  // exact
    bool ok = true;
    for (uint32_t t = 0; t < n; t++) {
        // Re(X_t * exp(-i pi t / n)) = re cos + im sin
        dd v = add(mul(re[t], dd{ch_[t], cl_[t]}), mul(im[t], dd{sh_[t], sl_[t]}));
        m[t] = round_away(mul_d(v, sc), ok);
    }
    (void)twon;
    return ok;
}

void Encoder::decode(const double *m, double scale, double *z, size_t nz) const
{
    const uint32_t n = n_;
    std::vector<std::complex<double>> a(n);
    for (uint32_t t = 0; t < n; t++) a[t] = std::complex<double>(m[t] * ch_[t], m[t] * sh_[t]);
    for (uint32_t i = 1, j = 0; i < n; i++) {
        uint32_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (uint32_t len = 2; len <= n; len <<= 1) {
        uint32_t h = len / 2, step = 2 * (n / len);
        for (uint32_t i = 0; i < n; i += len)
            for (uint32_t j = 0; j < h; j++) {
                uint32_t e = j * step;
                std::complex<double> w(ch_[e], sh_[e]);
                std::complex<double> u = a[i + j], v = a[i + j + h] * w;
                a[i + j] = u + v;
                a[i + j + h] = u - v;
            }
    }
    for (uint32_t j = 0; j < n / 2 && j < nz; j++) z[j] = a[slot_root_[j]].real() / scale;
}

}  // namespace hec
