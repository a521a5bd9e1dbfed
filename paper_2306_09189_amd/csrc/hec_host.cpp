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

// exp(x) for x <= 0 in double-double: x = k ln 2 + r (|r| <= ln2 / 2), exp(r / 2^8)
// by its Taylor series, squared eight times, scaled by 2^k
const dd LN2 = {6.931471805599452862e-01, 2.319046813846299558e-17};
dd exp_dd(dd x)
{
    const double k = std::nearbyint(x.h / LN2.h);
    dd r = sub(x, mul_d(LN2, k));
    r = {std::ldexp(r.h, -8), std::ldexp(r.l, -8)};
    dd term = {1.0, 0.0}, sum = term;
    for (int i = 1; i < 30; i++) {
        term = div_d(mul(term, r), (double)i);
        sum = add(sum, term);
        if (std::fabs(term.h) < 1e-40) break;
    }
    for (int i = 0; i < 8; i++) sum = mul(sum, sum);
    return {std::ldexp(sum.h, (int)k), std::ldexp(sum.l, (int)k)};
}
inline dd div_dd(dd a, dd b)
{
    double q1 = a.h / b.h;
    dd r = sub(a, mul_d(b, q1));
    double q2 = r.h / b.h;
    r = sub(r, mul_d(b, q2));
    double q3 = r.h / b.h;
    return add(quick(q1, q2), dd{q3, 0.0});
}
// floor of a non-negative double-double below 2^64
uint64_t floor_dd(dd x)
{
    const double fh = std::floor(x.h);
    dd f = two_sum(x.h - fh, x.l);  // x.h - fh is exact
    double ff = std::floor(f.h);
    if (ff == f.h && f.l < 0) ff -= 1;
    return (uint64_t)fh + (uint64_t)(int64_t)ff;
}

}  // namespace

// T[i] = floor(2^63 * sum_{|x| <= i} w(x) / sum_{|x| <= 19} w(x)), w(x) = exp(-x^2 / (2 sigma^2)),
// evaluated in double-double (about 100 bits): the thresholds of the table inversion sampler
bool gauss_table(double sigma, uint64_t T[19])
{
    if (!(sigma >= 2.0 && sigma <= 8.0)) return false;
    const dd den = mul_d(two_prod(sigma, sigma), 2.0);
    dd w[20], tot = {0.0, 0.0};
    for (int i = 0; i <= 19; i++) {
        w[i] = exp_dd(neg(div_dd(dd{(double)(i * i), 0.0}, den)));
        if (i) w[i] = mul_d(w[i], 2.0);
        tot = add(tot, w[i]);
    }
    dd acc = {0.0, 0.0};
    for (int i = 0; i < 19; i++) {
        acc = add(acc, w[i]);
        dd v = div_dd(acc, tot);
        T[i] = floor_dd({std::ldexp(v.h, 63), std::ldexp(v.l, 63)});
    }
    return true;
}

EncoderTables::EncoderTables(uint32_t logn)
{
    const uint32_t n = 1u << logn, twon = 2 * n;
    tw.resize(4 * (size_t)twon);
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
        tw[4 * (size_t)e] = C.h;
        tw[4 * (size_t)e + 1] = C.l;
        tw[4 * (size_t)e + 2] = S.h;
        tw[4 * (size_t)e + 3] = S.l;
    }
    root.resize(n / 2);
    uint64_t f = 1;
    for (uint32_t j = 0; j < n / 2; j++) {
        root[j] = (uint32_t)((f - 1) / 2);
        f = f * 5 % twon;
    }
}

}  // namespace hec
