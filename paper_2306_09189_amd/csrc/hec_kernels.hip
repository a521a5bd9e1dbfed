// hec_kernels.hip -- gfx950 kernels of the RNS-CKKS conv/pool library.
//
// Exact integer work on 64-bit prime limbs (all primes < 2^61):
//   * products by fixed constants (NTT twiddles, base-conversion and rescale
//     constants) use Shoup's precomputed quotient: q' = hi(a * w'), r = a*w - q'*q;
//   * products of two variables use Montgomery reduction with one operand
//     stored in Montgomery form (keys, plaintexts, public key);
//   * sums of several 128-bit products are accumulated exactly and reduced
//     once (base conversion, key-switch inner product).
// Everything runs on the VALU: this is exact modular arithmetic, not a float
// contraction, so the matrix cores are not used.
#include <atomic>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "hec_common.h"

#define DEV __device__ __forceinline__

// ---------------------------------------------------------------------------
// launch timing: while a kernel name is selected, every launch of that kernel
// is bracketed by HIP events on its stream and its work units are counted.
// ---------------------------------------------------------------------------
namespace {
struct Prof {
    char name[64] = {0};
    bool on = false;
    std::vector<hipEvent_t> pool, used;
    uint64_t launches = 0, units = 0;
};
Prof g_prof;
// launches of every named kernel since the library was loaded (counters are
// never freed, so a launch site keeps a pointer to its own)
std::mutex g_count_mu;
std::map<std::string, std::unique_ptr<std::atomic<uint64_t>>> g_count;
std::atomic<uint64_t> *prof_counter(const char *name)
{
    std::lock_guard<std::mutex> lk(g_count_mu);
    auto &p = g_count[name];
    if (!p) p.reset(new std::atomic<uint64_t>(0));
    return p.get();
}
hipEvent_t prof_event()
{
    hipEvent_t e;
    if (!g_prof.pool.empty()) {
        e = g_prof.pool.back();
        g_prof.pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        return nullptr;
    }
    g_prof.used.push_back(e);
    return e;
}
}  // namespace

void hec_prof_select(const char *name)
{
    for (auto e : g_prof.used) g_prof.pool.push_back(e);
    g_prof.used.clear();
    g_prof.launches = g_prof.units = 0;
    g_prof.on = name && name[0];
    if (g_prof.on) {
        strncpy(g_prof.name, name, sizeof(g_prof.name) - 1);
        g_prof.name[sizeof(g_prof.name) - 1] = 0;
    }
}
int hec_prof_collect(uint64_t *launches, uint64_t *units, double *ms)
{
    double tot = 0;
    for (size_t i = 0; i + 1 < g_prof.used.size(); i += 2) {
        if (hipEventSynchronize(g_prof.used[i + 1]) != hipSuccess) return -1;
        float t = 0;
        if (hipEventElapsedTime(&t, g_prof.used[i], g_prof.used[i + 1]) != hipSuccess) return -1;
        tot += t;
    }
    *launches = g_prof.launches;
    *units = g_prof.units;
    *ms = tot;
    return 0;
}
uint64_t hec_prof_count(const char *name)
{
    std::lock_guard<std::mutex> lk(g_count_mu);
    auto it = g_count.find(name);
    return it == g_count.end() ? 0 : it->second->load();
}
// A timed launch passes its events to the dispatch itself (hipExtLaunchKernelGGL),
// so the two timestamps bracket the kernel's execution and nothing else.
#define KLAUNCH(kname, nunits, kernel, grid, block, lds, st, ...)                                                  \
    do {                                                                                                           \
        static std::atomic<uint64_t> *cnt_ = prof_counter(kname);                                                  \
        cnt_->fetch_add(1, std::memory_order_relaxed);                                                             \
        if (g_prof.on && !strcmp(g_prof.name, kname)) {                                                            \
            hipEvent_t e0_ = prof_event(), e1_ = prof_event();                                                     \
            hipExtLaunchKernelGGL(kernel, grid, block, lds, st, e0_, e1_, 0, __VA_ARGS__);                        \
            g_prof.launches++;                                                                                     \
            g_prof.units += (nunits);                                                                              \
        } else {                                                                                                   \
            hipLaunchKernelGGL(kernel, grid, block, lds, st, __VA_ARGS__);                                         \
        }                                                                                                          \
    } while (0)

// ---------------------------------------------------------------------------
// modular helpers
// ---------------------------------------------------------------------------
DEV u64 add_mod(u64 a, u64 b, u64 q)
{
    u64 s = a + b;
    return s >= q ? s - q : s;
}
DEV u64 sub_mod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }
DEV u64 shoup_mul(u64 a, u64 w, u64 wsh, u64 q)
{
    u64 qt = __umul64hi(a, wsh);
    u64 r = a * w - qt * q;
    return r >= q ? r - q : r;
}
// T = hi:lo < q * 2^64  ->  T * 2^-64 mod q
DEV u64 redc(u64 hi, u64 lo, u64 q, u64 qinv_neg)
{
    u64 m = lo * qinv_neg;
    u64 r = hi + __umul64hi(m, q) + (lo != 0 ? 1 : 0);
    return r >= q ? r - q : r;
}
// 64 x 64 -> 128 bits from four 32 x 32 -> 64 products, each partial sum
// folded into the next product's addend (no carry is lost: a 32 x 32 product
// plus two 32-bit addends stays below 2^64).  The separate a * b and
// __umul64hi(a, b) would take six multiplies.
DEV void mul128(u64 a, u64 b, u64 &lo, u64 &hi)
{
    const u32 a0 = (u32)a, a1 = (u32)(a >> 32), b0 = (u32)b, b1 = (u32)(b >> 32);
    const u64 p00 = (u64)a0 * b0;
    const u64 t = (u64)a0 * b1 + (p00 >> 32);
    const u64 t2 = (u64)a1 * b0 + (u32)t;
    lo = (u64)(u32)p00 | (t2 << 32);
    hi = (u64)a1 * b1 + (t >> 32) + (t2 >> 32);
}
DEV u64 mont_mul(u64 a, u64 bm, u64 q, u64 qinv_neg)
{
    u64 lo, hi;
    mul128(a, bm, lo, hi);
    return redc(hi, lo, q, qinv_neg);
}
struct acc128 {
    u64 lo, hi;
};
DEV void mac(acc128 &acc, u64 a, u64 b)
{
    u64 lo, hi;
    mul128(a, b, lo, hi);
    acc.lo += lo;
    acc.hi += hi + (acc.lo < lo ? 1 : 0);
}
// Sums of up to 16 products a_i b_i with a_i, b_i < 2^60 (every prime here
// has at most 60 bits), exact, without a carry per product: each factor is
// split into 30-bit halves and the four partial products (each below 2^60) go
// to four 64-bit accumulators, which 16 of them cannot overflow.  One
// 32 x 32 -> 64 multiply-add per partial product; the 128-bit total is
// assembled once.  Same integer as the acc128 sum, so the same reduction.
struct acc30 {
    u64 s00, s01, s10, s11;
};
#define M30 0x3fffffffu
// x < 2^60 as the words (low 30 bits, high 30 bits)
DEV u64 split30(u64 x) { return (u64)((u32)x & M30) | ((x >> 30) << 32); }
DEV void mac30(acc30 &s, u64 a, u64 b)  // a, b as split30 gives them
{
    const u32 a0 = (u32)a, a1 = (u32)(a >> 32), b0 = (u32)b, b1 = (u32)(b >> 32);
    s.s00 += (u64)a0 * b0;
    s.s01 += (u64)a0 * b1;
    s.s10 += (u64)a1 * b0;
    s.s11 += (u64)a1 * b1;
}
// hi:lo = s00 + (s01 + s10) 2^30 + s11 2^60
DEV void acc30_total(const acc30 &s, u64 &lo, u64 &hi)
{
    const u64 m = s.s01 + s.s10;
    const u64 mc = m < s.s01 ? 1 : 0;  // the carry of m, weight 2^94
    const u64 t = m << 30;
    lo = s.s00 + t;
    hi = (m >> 34) + (mc << 30) + (lo < t ? 1 : 0);
    const u64 t2 = s.s11 << 60;
    lo += t2;
    hi += (s.s11 >> 4) + (lo < t2 ? 1 : 0);
}
DEV u32 brev_bits(u32 x, u32 bits) { return __brev(x) >> (32 - bits); }
// Evaluation-form index of sigma_g: slot k holds a(psi^(2 brv(k) + 1));
// sigma_g(a) at that root is a(psi^((2 brv(k)+1) g)).
DEV u32 auto_src(u32 k, u32 g, u32 logn)
{
    u32 n2 = 2u << logn;
    u32 e = 2 * brev_bits(k, logn) + 1;
    u32 eg = (u32)(((u64)e * g) & (n2 - 1));
    return brev_bits((eg - 1) >> 1, logn);
}

// ---------------------------------------------------------------------------
// NTT: merged Cooley-Tukey forward transform with bit-reversed output
// (a_hat[k] = a(psi^(2 brv(k) + 1))) and Gentleman-Sande inverse, split into a
// column pass (the first log2(n1) stages, strides >= n2) and a row pass (the
// last log2(n2) stages, inside rows of n2 contiguous words), each staged
// through LDS.  n = n1 * n2.
// ---------------------------------------------------------------------------
#define NTT_THREADS 256
#define NTT_TILE 4096  // words per LDS tile (32 KiB)

static inline void ntt_split(u32 logn, u32 &logn1, u32 &logn2)
{
    logn1 = logn / 2;
    logn2 = logn - logn1;
}

template <bool INV>
__global__ void __launch_bounds__(NTT_THREADS) k_ntt_cols(u64 *base, size_t poly_stride, const u32 *pmap, u32 logn,
                                                          u32 logn1, u32 C, DevTables T)
{
    extern __shared__ u64 lds[];
    const u32 limb = blockIdx.y;
    const u32 pi = pmap[limb];
    const u32 n2 = 1u << (logn - logn1), n1 = 1u << logn1;
    u64 *a = base + blockIdx.z * poly_stride + ((size_t)limb << logn);
    const u64 q = T.pc[pi].q;
    const u64 *w = (INV ? T.itw : T.tw) + ((size_t)pi << logn);
    const u64 *wsh = (INV ? T.itw_sh : T.tw_sh) + ((size_t)pi << logn);
    const u32 c0 = blockIdx.x * C;
    const u32 tile = n1 * C;
    for (u32 e = threadIdx.x; e < tile; e += NTT_THREADS) {
        u32 r = e / C, c = e % C;
        lds[e] = a[(size_t)r * n2 + c0 + c];
    }
    __syncthreads();
    const u32 nbf = (n1 / 2) * C;
    for (u32 st = 0; st < logn1; st++) {
        const u32 s = INV ? (logn1 - 1 - st) : st;  // global stage: m = 2^s
        const u32 m = 1u << s;
        const u32 tr = n1 >> (s + 1);
        for (u32 b = threadIdx.x; b < nbf; b += NTT_THREADS) {
            u32 c = b % C, bi = b / C;
            u32 grp = bi / tr, off = bi % tr;
            u32 r = grp * 2 * tr + off;
            u64 W = w[m + grp], Ws = wsh[m + grp];
            u64 *x = &lds[r * C + c], *y = &lds[(r + tr) * C + c];
            u64 U = *x, V = *y;
            if (!INV) {
                V = shoup_mul(V, W, Ws, q);
                *x = add_mod(U, V, q);
                *y = sub_mod(U, V, q);
            } else {
                *x = add_mod(U, V, q);
                *y = shoup_mul(sub_mod(U, V, q), W, Ws, q);
            }
        }
        __syncthreads();
    }
    if (INV) {
        const u64 ni = T.pc[pi].ninv, nis = T.pc[pi].ninv_sh;
        for (u32 e = threadIdx.x; e < tile; e += NTT_THREADS) {
            u32 r = e / C, c = e % C;
            a[(size_t)r * n2 + c0 + c] = shoup_mul(lds[e], ni, nis, q);
        }
    } else {
        for (u32 e = threadIdx.x; e < tile; e += NTT_THREADS) {
            u32 r = e / C, c = e % C;
            a[(size_t)r * n2 + c0 + c] = lds[e];
        }
    }
}

template <bool INV>
__global__ void __launch_bounds__(NTT_THREADS) k_ntt_rows(u64 *base, size_t poly_stride, const u32 *pmap, u32 logn,
                                                          u32 logn1, u32 R, DevTables T)
{
    extern __shared__ u64 lds[];
    const u32 limb = blockIdx.y;
    const u32 pi = pmap[limb];
    const u32 logn2 = logn - logn1;
    const u32 n2 = 1u << logn2;
    u64 *a = base + blockIdx.z * poly_stride + ((size_t)limb << logn) + (size_t)blockIdx.x * R * n2;
    const u64 q = T.pc[pi].q;
    const u64 *w = (INV ? T.itw : T.tw) + ((size_t)pi << logn);
    const u64 *wsh = (INV ? T.itw_sh : T.tw_sh) + ((size_t)pi << logn);
    const u32 r0 = blockIdx.x * R;
    const u32 tile = R * n2;
    for (u32 e = threadIdx.x; e < tile; e += NTT_THREADS) lds[e] = a[e];
    __syncthreads();
    const u32 half = n2 / 2, nbf = R * half;
    for (u32 st = 0; st < logn2; st++) {
        const u32 s2 = INV ? (logn2 - 1 - st) : st;
        const u32 m = 1u << (logn1 + s2);
        const u32 t = n2 >> (s2 + 1);
        for (u32 b = threadIdx.x; b < nbf; b += NTT_THREADS) {
            u32 row = b / half, bi = b % half;
            u32 grp = bi / t, off = bi % t;
            u32 c = grp * 2 * t + off;
            u32 widx = m + ((r0 + row) << s2) + grp;
            u64 W = w[widx], Ws = wsh[widx];
            u64 *x = &lds[row * n2 + c], *y = &lds[row * n2 + c + t];
            u64 U = *x, V = *y;
            if (!INV) {
                V = shoup_mul(V, W, Ws, q);
                *x = add_mod(U, V, q);
                *y = sub_mod(U, V, q);
            } else {
                *x = add_mod(U, V, q);
                *y = shoup_mul(sub_mod(U, V, q), W, Ws, q);
            }
        }
        __syncthreads();
    }
    for (u32 e = threadIdx.x; e < tile; e += NTT_THREADS) a[e] = lds[e];
}

// ---------------------------------------------------------------------------
// n = 2^16: both passes are 256-point transforms done as two radix-16 rounds
// (16 words per thread in registers, 4 stages per round, one LDS exchange per
// pass).  A tile is 16 transforms x 256 points: 16 columns in the column pass,
// 16 rows in the row pass.  Round A holds the points i + 16h (h = 0..15) of a
// transform, round B the points 16h + i.  Butterflies reduce lazily (Harvey):
// forward values stay in [0, 4q), inverse values in [0, 2q); outputs are
// fully reduced.
// ---------------------------------------------------------------------------
DEV u64 shoup_lazy(u64 a, u64 w, u64 wsh, u64 q) { return a * w - __umul64hi(a, wsh) * q; }  // [0, 2q)
DEV void ct_bfly(u64 &x, u64 &y, u64 W, u64 Ws, u64 q2, u64 q)
{
    u64 u = x >= q2 ? x - q2 : x;
    u64 v = shoup_lazy(y, W, Ws, q);
    x = u + v;
    y = u - v + q2;
}
DEV void gs_bfly(u64 &x, u64 &y, u64 W, u64 Ws, u64 q2, u64 q)
{
    u64 u = x, v = y;
    u64 s = u + v;
    x = s >= q2 ? s - q2 : s;
    y = shoup_lazy(u - v + q2, W, Ws, q);
}
DEV u64 reduce4(u64 x, u64 q)
{
    u64 q2 = 2 * q;
    x = x >= q2 ? x - q2 : x;
    return x >= q ? x - q : x;
}

// The arithmetic of the 2^16 transforms, in one of two exact forms:
//  * ArInt: 64-bit integers (any prime below 2^61), Shoup products by the
//    twiddles, values kept lazily in [0, 4q);
//  * ArFp: IEEE doubles, for primes below 2^50.  Every value is an integer
//    below 4q < 2^52, so it and every sum below are exact doubles.  The
//    product y w (y < 4q, w < q) is split exactly into ph + pl (ph = fl(y w),
//    pl = fma(y, w, -ph)); the quotient estimate k = floor(fl(y fl(w / q)))
//    differs from y w / q by less than 1 (both roundings below 2^-53
//    relative, y w / q < 2^52), so r = fma(-k, q, ph) + pl = y w - k q is an
//    exact integer in (-q, 2q) (|ph - k q| < 2q + 2^49 < 2^52 makes the fma
//    exact) and one conditional add puts it in [0, 2q).  That is the same
//    lazy range as the integer Shoup product, about half the instructions on
//    the VALU (the double multiply-add issues at the integer rate).
// Both keep the same ranges, so the canonical outputs -- and every bit that
// leaves a transform -- are the same.  Between the two passes the working
// values are stored in their own form (doubles as their bits).
struct ArInt {
    typedef u64 V;
    u64 q, q2;
    const u64 *w, *ws;  // twiddles psi^(+-brv(k)) (for the row pass: the first 128, staged in LDS)
    const u64 *z, *zs;  // row-pass twists
    DEV V in(u64 r) const { return r; }
    DEV V mid_in(u64 b) const { return b; }
    DEV u64 mid_out(V x) const { return x; }
    DEV void ct(V &x, V &y, u32 idx) const { ct_bfly(x, y, w[idx], ws[idx], q2, q); }
    DEV void gs(V &x, V &y, u32 idx) const { gs_bfly(x, y, w[idx], ws[idx], q2, q); }
    DEV V twist(V x, u32 k) const { return shoup_lazy(x, z[k], zs[k], q); }  // [0, 2q)
    DEV u64 full(V x) const { return reduce4(x, q); }  // [0, 4q) -> [0, q)
};
struct ArFp {
    typedef double V;
    double q, q2;
    const double2 *t;  // (w, fl(w / q)) (for the forward row pass: the first 128, staged in LDS)
    const double *tz;  // forward row-pass twists (words; their quotients by q rebuilt below)
    double qi;         // fl(1 / q)
    DEV V in(u64 r) const { return (double)r; }
    DEV V mid_in(u64 b) const { return __longlong_as_double((long long)b); }
    DEV u64 mid_out(V x) const { return (u64)__double_as_longlong(x); }
    DEV V mulmod(V y, double w, double wq) const
    {
        const double ph = y * w;
        const double pl = fma(y, w, -ph);
        const double k = floor(y * wq);
        const double r = fma(-k, q, ph) + pl;
        return r < 0.0 ? r + q : r;  // [0, 2q)
    }
    DEV void ct(V &x, V &y, u32 idx) const
    {
        const double2 tw = t[idx];
        const V u = x >= q2 ? x - q2 : x;
        const V v = mulmod(y, tw.x, tw.y);
        x = u + v;
        y = u - v + q2;
    }
    DEV void gs(V &x, V &y, u32 idx) const
    {
        const double2 tw = t[idx];
        const V u = x, v = y;
        const V s = u + v;
        x = s >= q2 ? s - q2 : s;
        y = mulmod(u - v + q2, tw.x, tw.y);
    }
    // x z_k, [0, 2q).  The quotient z / q is rebuilt from fl(1 / q) by one
    // residual step, e = z - fl(z / q)' q exactly (fma) and the quotient
    // corrected by e / q: within half an ulp plus 2^-104 relative of z / q,
    // inside what mulmod needs (its estimate of y z / q stays within 1 of the
    // truth for y < 4q < 2^52).
    DEV V twist(V x, u32 k) const
    {
        const double w = tz[k];
        const double w0 = w * qi;
        const double wq = fma(fma(-w0, q, w), qi, w0);
        return mulmod(x, w, wq);
    }
    DEV u64 full(V x) const
    {
        x = x >= q2 ? x - q2 : x;
        x = x >= q ? x - q : x;
        return (u64)x;
    }
};
DEV ArInt ar_int(const PrimeC &pc, const u64 *w, const u64 *ws, u32 pi)
{
    ArInt a;
    a.q = pc.q;
    a.q2 = 2 * pc.q;
    a.w = w + ((size_t)pi << 16);
    a.ws = ws + ((size_t)pi << 16);
    a.z = a.zs = nullptr;  // no twist outside the forward row pass
    return a;
}
DEV ArFp ar_fp(const PrimeC &pc, const double2 *t, u32 pi)
{
    ArFp a;
    a.q = pc.qd;
    a.q2 = 2.0 * pc.qd;
    a.t = t + ((size_t)pi << 16);
    a.tz = nullptr;  // no twist outside the forward row pass
    a.qi = pc.qinv_d;
    return a;
}
// LDS position of twiddle t in a row pass's table: one pad entry after every
// 8, so that the lanes of a row, which read entries 2^(s-4) apart in the
// second round of stage 8 + s, fall in different banks
#define RPAD(t) ((t) + ((t) >> 3))
#define RTAB 144  // entries of the padded table of 128
// the forward row pass's arithmetic: the twiddles psi^brv(t), t < 128, from
// their LDS copy bt (stage_row_twiddles), the twists of prime pi from HBM
DEV ArInt ar_int_rows(const PrimeC &pc, const u64 *bt, const u64 *z, const u64 *zs, u32 pi)
{
    ArInt a;
    a.q = pc.q;
    a.q2 = 2 * pc.q;
    a.w = bt;
    a.ws = bt + RTAB;
    a.z = z + ((size_t)pi << 16);
    a.zs = zs + ((size_t)pi << 16);
    return a;
}
DEV ArFp ar_fp_rows(const PrimeC &pc, const double2 *bt, const double *zf, u32 pi)
{
    ArFp a;
    a.q = pc.qd;
    a.q2 = 2.0 * pc.qd;
    a.t = bt;
    a.tz = zf + ((size_t)pi << 16);
    a.qi = pc.qinv_d;
    return a;
}
DEV bool use_fp(const DevTables &T, const PrimeC &pc) { return T.fp_on && pc.fp && T.twf; }
// the first CNT (<= 256) twiddles of prime pi in LDS (as (w, w / q) doubles,
// or as words followed by their Shoup companions), all lanes then
// synchronized: the 128 of a forward row pass (PAD: at RPAD(t), companions
// from RTAB on), the 256 of a column pass (in order, companions from CNT on)
template <int CNT, bool PAD>
DEV void stage_twiddles(bool fp, const u64 *w, const u64 *ws, const double2 *wf, u32 pi, double2 *bt)
{
    const u32 t = threadIdx.x;
    if (t < CNT) {
        const size_t at = ((size_t)pi << 16) + t;
        const u32 pos = PAD ? RPAD(t) : t;
        if (fp) {
            bt[pos] = wf[at];
        } else {
            ((u64 *)bt)[pos] = w[at];
            ((u64 *)bt)[(PAD ? RTAB : CNT) + pos] = ws[at];
        }
    }
    __syncthreads();
}
// the column passes' arithmetic with the twiddles of their LDS copy
DEV ArInt ar_int_lds(const PrimeC &pc, const u64 *bt, u32 cnt)
{
    ArInt a;
    a.q = pc.q;
    a.q2 = 2 * pc.q;
    a.w = bt;
    a.ws = bt + cnt;
    a.z = a.zs = nullptr;
    return a;
}
DEV ArFp ar_fp_lds(const PrimeC &pc, const double2 *bt)
{
    ArFp a;
    a.q = pc.qd;
    a.q2 = 2.0 * pc.qd;
    a.t = bt;
    a.tz = nullptr;
    a.qi = pc.qinv_d;
    return a;
}
// the tables as a launch of the 2^16 transforms sees them: the double
// butterflies on or off as the launch parameter says
static DevTables tuned(const DevTables &T)
{
    DevTables t = T;
    t.fp_on = hec_tune_params().ntt_fp64 ? 1u : 0u;
    return t;
}

#define N16_PAD(c) ((c) + ((c) >> 4))  // padded LDS index inside a 256-point row (17 words per 16)
DEV u64 mod64(u64 x, const PrimeC &pc);

// XCD-aware work order: workgroups are dealt round-robin to the 8 XCDs, each
// with its own L2.  The flat grid of 16 x nlimbs x npolys tiles is remapped so
// that each XCD walks one contiguous chunk of (limb, poly, tile) items; the
// polynomials that share a prime -- and its 1 MiB twiddle table -- then run
// back to back on the same L2 instead of being spread over all eight.
struct Ntt16Item {
    u32 tile, poly, limb;
};
// the same items in plain grid order (workgroups dealt to the XCDs round
// robin, so the chip works through the limbs in order)
DEV Ntt16Item ntt16_item_plain(u32 npolys)
{
    const u32 i = blockIdx.x;
    Ntt16Item it;
    it.tile = i & 15;
    const u32 rest = i >> 4;
    it.poly = rest % npolys;
    it.limb = rest / npolys;
    return it;
}
DEV Ntt16Item ntt16_item(u32 npolys)
{
    const u32 w = blockIdx.x, total = gridDim.x;  // total = 16 * nlimbs * npolys, a multiple of 8
    const u32 i = (w & 7) * (total >> 3) + (w >> 3);
    Ntt16Item it;
    it.tile = i & 15;
    const u32 rest = i >> 4;
    it.poly = rest % npolys;
    it.limb = rest / npolys;
    return it;
}

// forward column pass: stages 0..7 over the 256 rows of 16 columns (x holds
// the 16 points l + 16 h of column col, in the working form of Ar)
template <class Ar>
DEV void ntt16_fwd_cols_body(const Ar &ar, typename Ar::V *x, u64 *a, u64 *lds, u32 col, u32 l)
{
    typedef typename Ar::V V;
#pragma unroll
    for (int s = 0; s < 4; s++) {
        const int half = 8 >> s;
#pragma unroll
        for (int h = 0; h < 16; h++)
            if (!(h & half)) ar.ct(x[h], x[h + half], (1u << s) + (h >> (4 - s)));
    }
#pragma unroll
    for (int h = 0; h < 16; h++) lds[(l + 16 * h) * 16 + col] = ar.mid_out(x[h]);
    __syncthreads();
    const u32 hb = l;  // round B: rows 16*hb + i
    V y[16];
#pragma unroll
    for (int i = 0; i < 16; i++) y[i] = ar.mid_in(lds[(16 * hb + i) * 16 + col]);
#pragma unroll
    for (int s = 4; s < 8; s++) {
        const int half = 128 >> s;
#pragma unroll
        for (int i = 0; i < 16; i++)
            if (!(i & half)) ar.ct(y[i], y[i + half], (1u << s) + ((16 * hb + i) >> (8 - s)));
    }
#pragma unroll
    for (int i = 0; i < 16; i++) a[(size_t)(16 * hb + i) * 256 + col] = ar.mid_out(y[i]);
}

// (RS: the input is the centered dropped limb of a rescale, reduced mod this
// limb's prime)
template <bool RS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_ntt16_fwd_cols(u64 *base, size_t poly_stride, const u32 *pmap, u32 npolys,
                                                        RescaleFuse f, DevTables T)
{
    __shared__ u64 lds[256 * 16];
    __shared__ double2 bt[256];
    const Ntt16Item it = ntt16_item(npolys);
    const u32 pi = pmap[it.limb];
    const PrimeC pc = T.pc[pi];
    const u64 q = pc.q;
    u64 *a = base + it.poly * poly_stride + ((size_t)it.limb << 16) + it.tile * 16;
    const u32 col = threadIdx.x & 15, l = threadIdx.x >> 4;
    const bool fp = use_fp(T, pc);
    stage_twiddles<256, false>(fp, T.tw, T.tw_sh, T.twf, pi, bt);
    u64 r[16];
    if (RS) {
        const u64 ql = T.pc[f.level].q;
        const u64 *src = f.last + it.poly * f.ls + it.tile * 16;
#pragma unroll
        for (int h = 0; h < 16; h++) {
            const u64 v = src[(size_t)(l + 16 * h) * 256 + col];
            if (v <= (ql - 1) / 2) {
                r[h] = mod64(v, pc);
            } else {
                const u64 m = mod64(ql - v, pc);
                r[h] = m ? q - m : 0;
            }
        }
    } else {
#pragma unroll
        for (int h = 0; h < 16; h++) r[h] = a[(size_t)(l + 16 * h) * 256 + col];
    }
    if (fp) {
        const ArFp ar = ar_fp_lds(pc, bt);
        double x[16];
#pragma unroll
        for (int h = 0; h < 16; h++) x[h] = ar.in(r[h]);
        ntt16_fwd_cols_body(ar, x, a, lds, col, l);
    } else {
        ntt16_fwd_cols_body(ar_int_lds(pc, (const u64 *)bt, 256), r, a, lds, col, l);
    }
}

// forward row pass: stages 8..15 inside 16 rows of 256 words; the fully
// reduced output of each row is left in its LDS row lr (padded) for the
// epilogue of the caller
template <class Ar>
DEV void ntt16_fwd_rows_core(const Ar &ar, const u64 *a, u64 *lr, u32 grow, u32 row, u32 l)
{
    typedef typename Ar::V V;
    V x[16];
    // the row's twist R^c first (column c = l + 16 h); then the butterflies of
    // group t of every stage take the row-independent twiddle psi^brv16(t)
#pragma unroll
    for (int h = 0; h < 16; h++) x[h] = ar.twist(ar.mid_in(a[row * 256 + l + 16 * h]), grow * 256 + l + 16 * h);
#pragma unroll
    for (int s2 = 0; s2 < 4; s2++) {
        const int half = 8 >> s2;
#pragma unroll
        for (int h = 0; h < 16; h++)
            if (!(h & half)) ar.ct(x[h], x[h + half], RPAD(h >> (4 - s2)));
    }
#pragma unroll
    for (int h = 0; h < 16; h++) lr[N16_PAD(l + 16 * h)] = ar.mid_out(x[h]);
    __syncthreads();
    const u32 hb = l;
#pragma unroll
    for (int i = 0; i < 16; i++) x[i] = ar.mid_in(lr[N16_PAD(16 * hb + i)]);
#pragma unroll
    for (int s2 = 4; s2 < 8; s2++) {
        const int half = 128 >> s2;
#pragma unroll
        for (int i = 0; i < 16; i++)
            if (!(i & half)) ar.ct(x[i], x[i + half], RPAD((16 * hb + i) >> (8 - s2)));
    }
#pragma unroll
    for (int i = 0; i < 16; i++) lr[N16_PAD(16 * hb + i)] = ar.full(x[i]);
    __syncthreads();
}
// bt: 128 double2 of LDS for the staged twiddles
DEV void ntt16_fwd_rows_body(const DevTables &T, const PrimeC &pc, u32 pi, const u64 *a, u64 *lr, double2 *bt,
                             u32 grow, u32 row, u32 l)
{
    const bool fp = use_fp(T, pc);
    stage_twiddles<128, true>(fp, T.tw, T.tw_sh, T.twf, pi, bt);
    if (fp) ntt16_fwd_rows_core(ar_fp_rows(pc, bt, T.zf, pi), a, lr, grow, row, l);
    else ntt16_fwd_rows_core(ar_int_rows(pc, (const u64 *)bt, T.z, T.z_sh, pi), a, lr, grow, row, l);
}

// forward row pass; fully reduced output (RS: written as (c - output) q_l^-1
// to the rescaled polynomial)
template <bool RS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_ntt16_fwd_rows(u64 *base, size_t poly_stride, const u32 *pmap, u32 npolys,
                                                        RescaleFuse f, DevTables T)
{
    __shared__ u64 lds[16 * 272];
    __shared__ double2 bt[RTAB];
    const Ntt16Item it = ntt16_item(npolys);
    const u32 pi = pmap[it.limb];
    const PrimeC pc = T.pc[pi];
    const u64 q = pc.q;
    const u32 r0 = it.tile * 16;
    u64 *a = base + it.poly * poly_stride + ((size_t)it.limb << 16) + (size_t)r0 * 256;
    const u32 row = threadIdx.x >> 4, l = threadIdx.x & 15;
    u64 *lr = lds + row * 272;
    ntt16_fwd_rows_body(T, pc, pi, a, lr, bt, r0 + row, row, l);
    if (RS) {
        const size_t off = ((size_t)it.limb << 16) + (size_t)r0 * 256 + row * 256;
        const u64 *cp = f.c + it.poly * f.cs + off;
        u64 *op = f.out + it.poly * f.os + off;
        const u64 qi = f.lc->qlinv[it.limb], qis = f.lc->qlinv_sh[it.limb];
#pragma unroll
        for (int h = 0; h < 16; h++)
            op[l + 16 * h] = shoup_mul(sub_mod(cp[l + 16 * h], lr[N16_PAD(l + 16 * h)], q), qi, qis, q);
    } else {
#pragma unroll
        for (int h = 0; h < 16; h++) a[row * 256 + l + 16 * h] = lr[N16_PAD(l + 16 * h)];
    }
}

// Forward row pass with 8 values per lane: 512 lanes per 16-row tile, 32 per
// row, radix-8, radix-8 and radix-4 rounds with two LDS exchanges.  Half the
// registers of the 16-value form, so up to twice the waves per SIMD to cover
// the memory latency.  Same butterflies (the twist, then twiddle psi^brv16(t)
// for group t = c >> (8 - s) of stage 8 + s), same residues.  Leaves the fully
// reduced values of columns 4 (l + 32 g) + i (g < 2, i < 4) in y[4 g + i].
template <class Ar>
DEV void ntt16_fwd_rows_core8(const Ar &ar, const u64 *a, u64 *lr, u32 grow, u32 l, u64 *y)
{
    typedef typename Ar::V V;
    V x[8];
#pragma unroll
    for (int h = 0; h < 8; h++) x[h] = ar.twist(ar.mid_in(a[l + 32 * h]), grow * 256 + l + 32 * h);
#pragma unroll
    for (int s2 = 0; s2 < 3; s2++) {  // columns l + 32 h
        const int half = 4 >> s2;
#pragma unroll
        for (int h = 0; h < 8; h++)
            if (!(h & half)) ar.ct(x[h], x[h + half], RPAD(h >> (3 - s2)));
    }
#pragma unroll
    for (int h = 0; h < 8; h++) lr[N16_PAD(l + 32 * h)] = ar.mid_out(x[h]);
    __syncthreads();
    const u32 cb = 32 * (l >> 2) + (l & 3);  // columns cb + 4 j: each read by this lane alone,
#pragma unroll                              // so it may overwrite them without a barrier
    for (int j = 0; j < 8; j++) x[j] = ar.mid_in(lr[N16_PAD(cb + 4 * j)]);
#pragma unroll
    for (int s2 = 3; s2 < 6; s2++) {
        const int half = 4 >> (s2 - 3);
#pragma unroll
        for (int j = 0; j < 8; j++)
            if (!(j & half)) ar.ct(x[j], x[j + half], RPAD((cb + 4 * j) >> (8 - s2)));
    }
#pragma unroll
    for (int j = 0; j < 8; j++) lr[N16_PAD(cb + 4 * j)] = ar.mid_out(x[j]);
    __syncthreads();
#pragma unroll
    for (int g = 0; g < 2; g++) {  // columns 4 m + i, m = l + 32 g
        const u32 m = l + 32 * g;
#pragma unroll
        for (int i = 0; i < 4; i++) x[4 * g + i] = ar.mid_in(lr[N16_PAD(4 * m + i)]);
        ar.ct(x[4 * g], x[4 * g + 2], RPAD(m));
        ar.ct(x[4 * g + 1], x[4 * g + 3], RPAD(m));
        ar.ct(x[4 * g], x[4 * g + 1], RPAD(2 * m));
        ar.ct(x[4 * g + 2], x[4 * g + 3], RPAD(2 * m + 1));
    }
#pragma unroll
    for (int k = 0; k < 8; k++) y[k] = ar.full(x[k]);
}
DEV void ntt16_fwd_rows_body8(const DevTables &T, const PrimeC &pc, u32 pi, const u64 *a, u64 *lr, double2 *bt,
                              u32 grow, u32 l, u64 *y)
{
    const bool fp = use_fp(T, pc);
    stage_twiddles<128, true>(fp, T.tw, T.tw_sh, T.twf, pi, bt);
    if (fp) ntt16_fwd_rows_core8(ar_fp_rows(pc, bt, T.zf, pi), a, lr, grow, l, y);
    else ntt16_fwd_rows_core8(ar_int_rows(pc, (const u64 *)bt, T.z, T.z_sh, pi), a, lr, grow, l, y);
}
// column of value k of a lane in the 8-value row pass
#define R8_COL(l, k) (4 * ((l) + 32 * ((k) >> 2)) + ((k) & 3))

template <bool RS>
__global__ void __launch_bounds__(512) k_ntt16_fwd_rows8(u64 *base, size_t poly_stride, const u32 *pmap,
                                                         u32 npolys, RescaleFuse f, DevTables T)
{
    __shared__ u64 lds[16 * 272];
    __shared__ double2 bt[RTAB];
    const Ntt16Item it = ntt16_item(npolys);
    const u32 pi = pmap[it.limb];
    const PrimeC pc = T.pc[pi];
    const u64 q = pc.q;
    const u32 r0 = it.tile * 16;
    const u32 row = threadIdx.x >> 5, l = threadIdx.x & 31;
    u64 *a = base + it.poly * poly_stride + ((size_t)it.limb << 16) + (size_t)(r0 + row) * 256;
    u64 y[8];
    ntt16_fwd_rows_body8(T, pc, pi, a, lds + row * 272, bt, r0 + row, l, y);
    if (RS) {
        const size_t off = ((size_t)it.limb << 16) + (size_t)(r0 + row) * 256;
        const u64 *cp = f.c + it.poly * f.cs + off;
        u64 *op = f.out + it.poly * f.os + off;
        const u64 qi = f.lc->qlinv[it.limb], qis = f.lc->qlinv_sh[it.limb];
#pragma unroll
        for (int k = 0; k < 8; k++) op[R8_COL(l, k)] = shoup_mul(sub_mod(cp[R8_COL(l, k)], y[k], q), qi, qis, q);
    } else {
#pragma unroll
        for (int k = 0; k < 8; k++) a[R8_COL(l, k)] = y[k];
    }
}
__global__ void __launch_bounds__(512) k_ntt16_fwd_rows8_md(u64 *yb, u32 nq, u32 nqp, const u32 *pmap, u32 npolys,
                                                            CombineBatch cb, const LevelC *lc, DevTables T)
{
    __shared__ u64 lds[16 * 272];
    __shared__ double2 bt[RTAB];
    const Ntt16Item it = ntt16_item(npolys);
    const u32 pi = pmap[it.limb];
    const PrimeC pc = T.pc[pi];
    const u64 q = pc.q;
    const u32 r0 = it.tile * 16;
    const u32 row = threadIdx.x >> 5, l = threadIdx.x & 31;
    const size_t ps = (size_t)nq << 16;
    const u64 *a = yb + it.poly * ps + ((size_t)it.limb << 16) + (size_t)(r0 + row) * 256;
    u64 y[8];
    ntt16_fwd_rows_body8(T, pc, pi, a, lds + row * 272, bt, r0 + row, l, y);
    const u32 r = it.poly >> 1, p = it.poly & 1, i = it.limb;
    if (!cb.out[r]) return;  // a slot of the batch nobody asked for
    const u64 pinv = lc->pinv[i], pinv_sh = lc->pinv_sh[i];
    const size_t ro = (size_t)(r0 + row) * 256;
    const u64 *e = cb.e[r] + ((size_t)p * nqp + i) * 65536 + ro;
    u64 *out = cb.out[r] + ((size_t)p * nq + i) * 65536 + ro;
    const u64 *c0 = (p == 0 && cb.c0[r]) ? cb.c0[r] + (size_t)i * 65536 : nullptr;
    const u64 *ad = cb.add[r][p] ? cb.add[r][p] + (size_t)i * 65536 + ro : nullptr;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const u32 c = R8_COL(l, k);
        u64 v = shoup_mul(sub_mod(e[c], y[k], q), pinv, pinv_sh, q);
        if (c0) v = add_mod(v, c0[auto_src((u32)ro + c, cb.g[r], 16)], q);
        if (ad) v = add_mod(v, ad[c], q);
        out[c] = v;
    }
}

// forward row pass of the P -> Q conversion y of a batch of ModDowns (poly z
// = entry z / 2, polynomial z % 2) with the ModDown tail as its epilogue:
// out = (e - NTT(y)) P^-1 (+ sigma_g(c0) on polynomial 0, + add), so NTT(y) is
// never written back and read again.  Same residues as the row pass followed
// by k_moddown_combine.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_ntt16_fwd_rows_md(u64 *y, u32 nq, u32 nqp, const u32 *pmap, u32 npolys, CombineBatch cb, const LevelC *lc,
                    DevTables T)
{
    __shared__ u64 lds[16 * 272];
    __shared__ double2 bt[RTAB];
    // plain order: the rotated ciphertexts are written limb by limb across the
    // chip, and the weight products that follow walk the limbs from the top,
    // so they start with the last-written ones (the two orders together took
    // 0.7 % off the benchmark step against the XCD-contiguous order here)
    const Ntt16Item it = ntt16_item_plain(npolys);
    const u32 pi = pmap[it.limb];
    const PrimeC pc = T.pc[pi];
    const u64 q = pc.q;
    const u32 r0 = it.tile * 16;
    const size_t ps = (size_t)nq << 16;
    u64 *a = y + it.poly * ps + ((size_t)it.limb << 16) + (size_t)r0 * 256;
    const u32 row = threadIdx.x >> 4, l = threadIdx.x & 15;
    u64 *lr = lds + row * 272;
    ntt16_fwd_rows_body(T, pc, pi, a, lr, bt, r0 + row, row, l);
    const u32 r = it.poly >> 1, p = it.poly & 1, i = it.limb;
    if (!cb.out[r]) return;  // a slot of the batch nobody asked for
    const u64 pinv = lc->pinv[i], pinv_sh = lc->pinv_sh[i];
    const u64 *e = cb.e[r] + ((size_t)p * nqp + i) * 65536;
    u64 *out = cb.out[r] + ((size_t)p * nq + i) * 65536;
    const u64 *c0 = (p == 0 && cb.c0[r]) ? cb.c0[r] + (size_t)i * 65536 : nullptr;
    const u64 *ad = cb.add[r][p] ? cb.add[r][p] + (size_t)i * 65536 : nullptr;
#pragma unroll
    for (int h = 0; h < 16; h++) {
        const u32 k = (r0 + row) * 256 + l + 16 * h;
        u64 v = shoup_mul(sub_mod(e[k], lr[N16_PAD(l + 16 * h)], q), pinv, pinv_sh, q);
        if (c0) v = add_mod(v, c0[auto_src(k, cb.g[r], 16)], q);
        if (ad) v = add_mod(v, ad[k], q);
        out[k] = v;
    }
}

// inverse row pass: stages 15..8 (Gentleman-Sande) inside 16 rows (OOP: the
// input read from src with its own poly stride, the output written to base)
template <class Ar>
DEV void ntt16_inv_rows_core(const Ar &ar, const u64 *in, u64 *a, u64 *lr, u32 grow, u32 row, u32 l)
{
    typedef typename Ar::V V;
    V x[16];
#pragma unroll
    for (int h = 0; h < 16; h++) lr[N16_PAD(l + 16 * h)] = in[row * 256 + l + 16 * h];
    __syncthreads();
    const u32 hb = l;
#pragma unroll
    for (int i = 0; i < 16; i++) x[i] = ar.in(lr[N16_PAD(16 * hb + i)]);
#pragma unroll
    for (int s2 = 7; s2 >= 4; s2--) {
        const int half = 128 >> s2;
#pragma unroll
        for (int i = 0; i < 16; i++)
            if (!(i & half)) ar.gs(x[i], x[i + half], (256u << s2) + (grow << s2) + ((16 * hb + i) >> (8 - s2)));
    }
#pragma unroll
    for (int i = 0; i < 16; i++) lr[N16_PAD(16 * hb + i)] = ar.mid_out(x[i]);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 16; h++) x[h] = ar.mid_in(lr[N16_PAD(l + 16 * h)]);
#pragma unroll
    for (int s2 = 3; s2 >= 0; s2--) {
        const int half = 8 >> s2;
#pragma unroll
        for (int h = 0; h < 16; h++)
            if (!(h & half)) ar.gs(x[h], x[h + half], (256u << s2) + (grow << s2) + (h >> (4 - s2)));
    }
#pragma unroll
    for (int h = 0; h < 16; h++) a[row * 256 + l + 16 * h] = ar.mid_out(x[h]);
}
template <bool OOP>
__global__ void __launch_bounds__(256) k_ntt16_inv_rows(u64 *base, size_t poly_stride, const u32 *pmap, u32 npolys,
                                                        const u64 *src, size_t src_stride, DevTables T)
{
    __shared__ u64 lds[16 * 272];
    const Ntt16Item it = ntt16_item(npolys);
    const u32 pi = pmap[it.limb];
    const PrimeC pc = T.pc[pi];
    const u32 r0 = it.tile * 16;
    u64 *a = base + it.poly * poly_stride + ((size_t)it.limb << 16) + (size_t)r0 * 256;
    const u32 row = threadIdx.x >> 4, l = threadIdx.x & 15;
    u64 *lr = lds + row * 272;
    const u64 *in = OOP ? src + it.poly * src_stride + ((size_t)it.limb << 16) + (size_t)r0 * 256 : a;
    if (use_fp(T, pc)) ntt16_inv_rows_core(ar_fp(pc, T.itwf, pi), in, a, lr, r0 + row, row, l);
    else ntt16_inv_rows_core(ar_int(pc, T.itw, T.itw_sh, pi), in, a, lr, r0 + row, row, l);
}

// inverse column pass: stages 7..0, then the factor n^-1; fully reduced output
template <class Ar>
DEV void ntt16_inv_cols_core(const Ar &ar, u64 *a, u64 *lds, u32 col, u32 l, const PrimeC &pc);
DEV u64 ninv_full(const ArInt &ar, u64 x, const PrimeC &pc) { return shoup_mul(x, pc.ninv, pc.ninv_sh, pc.q); }
DEV u64 ninv_full(const ArFp &ar, double x, const PrimeC &pc)
{
    double r = ar.mulmod(x, (double)pc.ninv, pc.ninv_q);  // [0, 2q)
    r = r >= ar.q ? r - ar.q : r;
    return (u64)r;
}
template <class Ar>
DEV void ntt16_inv_cols_core(const Ar &ar, u64 *a, u64 *lds, u32 col, u32 l, const PrimeC &pc)
{
    typedef typename Ar::V V;
    const u32 hb = l;
    V x[16];
#pragma unroll
    for (int i = 0; i < 16; i++) x[i] = ar.mid_in(a[(size_t)(16 * hb + i) * 256 + col]);
#pragma unroll
    for (int s = 7; s >= 4; s--) {
        const int half = 128 >> s;
#pragma unroll
        for (int i = 0; i < 16; i++)
            if (!(i & half)) ar.gs(x[i], x[i + half], (1u << s) + ((16 * hb + i) >> (8 - s)));
    }
#pragma unroll
    for (int i = 0; i < 16; i++) lds[(16 * hb + i) * 16 + col] = ar.mid_out(x[i]);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 16; h++) x[h] = ar.mid_in(lds[(l + 16 * h) * 16 + col]);
#pragma unroll
    for (int s = 3; s >= 0; s--) {
        const int half = 8 >> s;
#pragma unroll
        for (int h = 0; h < 16; h++)
            if (!(h & half)) ar.gs(x[h], x[h + half], (1u << s) + (h >> (4 - s)));
    }
#pragma unroll
    for (int h = 0; h < 16; h++) a[(size_t)(l + 16 * h) * 256 + col] = ninv_full(ar, x[h], pc);
}
__global__ void __launch_bounds__(256) k_ntt16_inv_cols(u64 *base, size_t poly_stride, const u32 *pmap, u32 npolys,
                                                        DevTables T)
{
    __shared__ u64 lds[256 * 16];
    const Ntt16Item it = ntt16_item(npolys);
    const u32 pi = pmap[it.limb];
    const PrimeC pc = T.pc[pi];
    u64 *a = base + it.poly * poly_stride + ((size_t)it.limb << 16) + it.tile * 16;
    const u32 col = threadIdx.x & 15, l = threadIdx.x >> 4;
    if (use_fp(T, pc)) ntt16_inv_cols_core(ar_fp(pc, T.itwf, pi), a, lds, col, l, pc);
    else ntt16_inv_cols_core(ar_int(pc, T.itw, T.itw_sh, pi), a, lds, col, l, pc);
}

TuneParams &hec_tune_params()
{
    static TuneParams p;
    return p;
}
static void ntt_launch_one(const DevTables &T, bool inv, u64 *base, size_t poly_stride, int npolys, const u32 *pmap,
                           int nlimbs, hipStream_t st);

static void ntt_launch(const DevTables &T, bool inv, u64 *base, size_t poly_stride, int npolys, const u32 *pmap,
                       int nlimbs, hipStream_t st)
{
    if (nlimbs <= 0 || npolys <= 0) return;
    const TuneParams &tp = hec_tune_params();
    // limb grouping: several launches of at most ntt_group limbs each
    if (tp.ntt_group > 0 && (int64_t)nlimbs * npolys > tp.ntt_group) {
        if (nlimbs > tp.ntt_group) {
            for (int p = 0; p < npolys; p++)
                for (int l0 = 0; l0 < nlimbs; l0 += tp.ntt_group)
                    ntt_launch_one(T, inv, base + (size_t)p * poly_stride + (size_t)l0 * T.n, poly_stride, 1,
                                   pmap + l0, std::min(tp.ntt_group, nlimbs - l0), st);
        } else {
            const int per = tp.ntt_group / nlimbs;
            for (int p0 = 0; p0 < npolys; p0 += per)
                ntt_launch_one(T, inv, base + (size_t)p0 * poly_stride, poly_stride, std::min(per, npolys - p0), pmap,
                               nlimbs, st);
        }
        return;
    }
    ntt_launch_one(T, inv, base, poly_stride, npolys, pmap, nlimbs, st);
}

static void ntt_launch_one(const DevTables &T, bool inv, u64 *base, size_t poly_stride, int npolys, const u32 *pmap,
                           int nlimbs, hipStream_t st)
{
    const TuneParams &tp = hec_tune_params();
    if (T.logn == 16 && tp.ntt16_radix == 16) {
        const uint64_t limbs = (uint64_t)nlimbs * npolys;
        dim3 g((u32)(16 * limbs));
        const u32 np = (u32)npolys;
        if (!inv) {
            KLAUNCH("k_ntt16_fwd_cols", limbs, k_ntt16_fwd_cols<false>, g, dim3(256), 0, st, base, poly_stride, pmap,
                    np, RescaleFuse{}, tuned(T));
            // units of the row pass: 2^16-word limbs read or written (here one of each per limb)
            if (tp.ntt_row_vals == 8)
                KLAUNCH("k_ntt16_fwd_rows", 2 * limbs, k_ntt16_fwd_rows8<false>, g, dim3(512), 0, st, base,
                        poly_stride, pmap, np, RescaleFuse{}, tuned(T));
            else
                KLAUNCH("k_ntt16_fwd_rows", 2 * limbs, k_ntt16_fwd_rows<false>, g, dim3(256), 0, st, base,
                        poly_stride, pmap, np, RescaleFuse{}, tuned(T));
        } else {
            KLAUNCH("k_ntt16_inv_rows", limbs, k_ntt16_inv_rows<false>, g, dim3(256), 0, st, base, poly_stride, pmap,
                    np, nullptr, (size_t)0, tuned(T));
            KLAUNCH("k_ntt16_inv_cols", limbs, k_ntt16_inv_cols, g, dim3(256), 0, st, base, poly_stride, pmap, np, tuned(T));
        }
        return;
    }
    u32 logn1, logn2;
    ntt_split(T.logn, logn1, logn2);
    u32 n1 = 1u << logn1, n2 = 1u << logn2;
    u32 C = n2 < 16 ? n2 : 16;
    const u32 tile = (tp.ntt_tile == 2048 || tp.ntt_tile == 8192) ? (u32)tp.ntt_tile : NTT_TILE;
    u32 R = tile / n2;
    if (R > n1) R = n1;
    if (R < 1) R = 1;
    dim3 gc(n2 / C, nlimbs, npolys), gr(n1 / R, nlimbs, npolys);
    size_t lc = (size_t)n1 * C * 8, lr = (size_t)R * n2 * 8;
    if (!inv) {
        hipLaunchKernelGGL(k_ntt_cols<false>, gc, dim3(NTT_THREADS), lc, st, base, poly_stride, pmap, T.logn, logn1,
                           C, T);
        hipLaunchKernelGGL(k_ntt_rows<false>, gr, dim3(NTT_THREADS), lr, st, base, poly_stride, pmap, T.logn, logn1,
                           R, T);
    } else {
        hipLaunchKernelGGL(k_ntt_rows<true>, gr, dim3(NTT_THREADS), lr, st, base, poly_stride, pmap, T.logn, logn1, R,
                           T);
        hipLaunchKernelGGL(k_ntt_cols<true>, gc, dim3(NTT_THREADS), lc, st, base, poly_stride, pmap, T.logn, logn1, C,
                           T);
    }
}

bool hec_ntt_inv_from(const DevTables &T, u64 *dst, size_t dst_stride, const u64 *src, size_t src_stride,
                      int npolys, const u32 *pmap, int nlimbs, hipStream_t st)
{
    if (T.logn != 16 || npolys <= 0 || nlimbs <= 0) return false;
    const uint64_t limbs = (uint64_t)nlimbs * npolys;
    dim3 g((u32)(16 * limbs));
    const u32 np = (u32)npolys;
    KLAUNCH("k_ntt16_inv_rows", limbs, k_ntt16_inv_rows<true>, g, dim3(256), 0, st, dst, dst_stride, pmap, np, src,
            src_stride, tuned(T));
    KLAUNCH("k_ntt16_inv_cols", limbs, k_ntt16_inv_cols, g, dim3(256), 0, st, dst, dst_stride, pmap, np, tuned(T));
    return true;
}
bool hec_ntt_fwd_moddown(const DevTables &T, u64 *y, int nrot, int nq, int nqp, const CombineBatch &cb,
                         const LevelC *lc, const u32 *pmap, hipStream_t st)
{
    if (T.logn != 16 || nrot < 1 || nrot > HEC_ROT_BATCH || nq < 1) return false;
    const u32 np = 2u * (u32)nrot;
    const uint64_t limbs = (uint64_t)nq * np;
    dim3 g((u32)(16 * limbs));
    KLAUNCH("k_ntt16_fwd_cols", limbs, k_ntt16_fwd_cols<false>, g, dim3(256), 0, st, y, (size_t)nq << 16, pmap, np,
            RescaleFuse{}, tuned(T));
    // limbs moved: y read; for every entry asked for, e read and the output written, sigma_g(c0)
    // read on polynomial 0 and the added polynomials read
    uint64_t units = 0;
    for (int r = 0; r < nrot; r++)
        for (int p = 0; p < 2; p++)
            units += (uint64_t)nq * (cb.out[r] ? 3 + (p == 0 && cb.c0[r] ? 1 : 0) + (cb.add[r][p] ? 1 : 0) : 1);
    if (hec_tune_params().ntt_row_vals == 8)
        KLAUNCH("k_ntt16_fwd_rows", units, k_ntt16_fwd_rows8_md, g, dim3(512), 0, st, y, (u32)nq, (u32)nqp, pmap, np,
                cb, lc, tuned(T));
    else
        KLAUNCH("k_ntt16_fwd_rows", units, k_ntt16_fwd_rows_md, g, dim3(256), 0, st, y, (u32)nq, (u32)nqp, pmap, np,
                cb, lc, tuned(T));
    return true;
}
bool hec_ntt_fwd_rescale(const DevTables &T, u64 *tmp, int npolys, const u32 *pmap, const RescaleFuse &f,
                         hipStream_t st)
{
    if (T.logn != 16 || npolys <= 0 || f.level == 0) return false;
    const u32 l = f.level;
    const uint64_t limbs = (uint64_t)l * npolys;
    dim3 g((u32)(16 * limbs));
    const size_t ps = (size_t)l << 16;
    const u32 np = (u32)npolys;
    KLAUNCH("k_ntt16_fwd_cols", limbs, k_ntt16_fwd_cols<true>, g, dim3(256), 0, st, tmp, ps, pmap, np, f, tuned(T));
    // limbs moved: the transformed limb and c read, the rescaled limb written
    if (hec_tune_params().ntt_row_vals == 8)
        KLAUNCH("k_ntt16_fwd_rows", 3 * limbs, k_ntt16_fwd_rows8<true>, g, dim3(512), 0, st, tmp, ps, pmap, np, f,
                tuned(T));
    else
        KLAUNCH("k_ntt16_fwd_rows", 3 * limbs, k_ntt16_fwd_rows<true>, g, dim3(256), 0, st, tmp, ps, pmap, np, f,
                tuned(T));
    return true;
}
void hec_ntt_fwd(const DevTables &T, u64 *base, size_t poly_stride, int npolys, const u32 *pmap, int nlimbs,
                 hipStream_t st)
{
    ntt_launch(T, false, base, poly_stride, npolys, pmap, nlimbs, st);
}
void hec_ntt_inv(const DevTables &T, u64 *base, size_t poly_stride, int npolys, const u32 *pmap, int nlimbs,
                 hipStream_t st)
{
    ntt_launch(T, true, base, poly_stride, npolys, pmap, nlimbs, st);
}

// ---------------------------------------------------------------------------
// elementwise
// ---------------------------------------------------------------------------
#define EW_THREADS 256
__global__ void __launch_bounds__(EW_THREADS) k_ew(int op, u64 *out, const u64 *a, const u64 *b, size_t so, size_t sa,
                                                   size_t sb, const u32 *pmap, DevTables T)
{
    const u32 limb = blockIdx.y, p = blockIdx.z;
    const PrimeC pc = T.pc[pmap[limb]];
    const size_t n = T.n;
    const size_t t = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (t >= n) return;
    const size_t off = (size_t)limb * n + t;
    u64 *o = out + p * so + off;
    const u64 *x = a ? a + p * sa + off : nullptr;
    const u64 *y = b ? b + p * sb + off : nullptr;
    switch (op) {
    case EW_ADD: *o = add_mod(*x, *y, pc.q); break;
    case EW_SUB: *o = sub_mod(*x, *y, pc.q); break;
    case EW_NEG: *o = *x ? pc.q - *x : 0; break;
    case EW_MUL_MONT: *o = mont_mul(*x, *y, pc.q, pc.qinv_neg); break;
    case EW_MAC_MONT: *o = add_mod(*o, mont_mul(*x, *y, pc.q, pc.qinv_neg), pc.q); break;
    case EW_TO_MONT: *o = mont_mul(*x, pc.r2, pc.q, pc.qinv_neg); break;
    case EW_FROM_MONT: *o = redc(0, *x, pc.q, pc.qinv_neg); break;
    case EW_COPY: *o = *x; break;
    case EW_ZERO: *o = 0; break;
    case EW_DBL_SUB: *o = sub_mod(add_mod(*x, *x, pc.q), *y, pc.q); break;
    }
}

void hec_ew(const DevTables &T, EwOp op, u64 *out, const u64 *a, const u64 *b, size_t so, size_t sa, size_t sb,
            int npolys, const u32 *pmap, int nlimbs, hipStream_t st)
{
    if (nlimbs <= 0 || npolys <= 0) return;
    dim3 g((T.n + EW_THREADS - 1) / EW_THREADS, nlimbs, npolys);
    KLAUNCH("k_ew", (uint64_t)npolys * nlimbs, k_ew, g, dim3(EW_THREADS), 0, st, (int)op, out, a, b, so, sa, sb, pmap,
            T);
}

__global__ void k_reduce_i64(u64 *out, const int64_t *x, const u32 *pmap, DevTables T)
{
    const u32 limb = blockIdx.y;
    const size_t t = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (t >= T.n) return;
    const u64 q = T.pc[pmap[limb]].q;
    int64_t v = x[t];
    u64 r;
    if (v >= 0) r = (u64)v % q;
    else {
        u64 m = ((u64)(-(v + 1)) + 1) % q;
        r = m ? q - m : 0;
    }
    out[(size_t)limb * T.n + t] = r;
}

void hec_reduce_i64(const DevTables &T, u64 *out, const int64_t *x, const u32 *pmap, int nlimbs, hipStream_t st)
{
    dim3 g((T.n + EW_THREADS - 1) / EW_THREADS, nlimbs, 1);
    hipLaunchKernelGGL(k_reduce_i64, g, dim3(EW_THREADS), 0, st, out, x, pmap, T);
}

__global__ void k_copy_limbs(u64 *dst, const u64 *src, size_t dps, size_t sps, size_t elems)
{
    size_t i = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (i >= elems) return;
    dst[blockIdx.y * dps + i] = src[blockIdx.y * sps + i];
}
void hec_copy_limbs(u64 *dst, const u64 *src, size_t dst_poly_stride, size_t src_poly_stride, int npolys,
                    size_t limb_elems, hipStream_t st)
{
    if (!limb_elems || npolys <= 0) return;
    dim3 g((limb_elems + EW_THREADS - 1) / EW_THREADS, npolys, 1);
    hipLaunchKernelGGL(k_copy_limbs, g, dim3(EW_THREADS), 0, st, dst, src, dst_poly_stride, src_poly_stride,
                       limb_elems);
}

__global__ void k_automorph(u64 *out, const u64 *in, size_t ps, u32 g, DevTables T)
{
    const u32 limb = blockIdx.y, p = blockIdx.z;
    const u32 k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= T.n) return;
    const size_t off = p * ps + (size_t)limb * T.n;
    out[off + k] = in[off + auto_src(k, g, T.logn)];
}
void hec_automorph_ntt(const DevTables &T, u64 *out, const u64 *in, size_t poly_stride, int npolys, int nlimbs,
                       u32 g, hipStream_t st)
{
    dim3 gr((T.n + EW_THREADS - 1) / EW_THREADS, nlimbs, npolys);
    hipLaunchKernelGGL(k_automorph, gr, dim3(EW_THREADS), 0, st, out, in, poly_stride, g, T);
}

// ---------------------------------------------------------------------------
// ChaCha20 (RFC 8439) and samplers
// ---------------------------------------------------------------------------
DEV u32 rotl(u32 x, int r) { return (x << r) | (x >> (32 - r)); }
DEV void chacha_block(u64 seed, u32 purpose, u64 index, u32 counter, u32 out[16])
{
    u32 s[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u, (u32)seed, (u32)(seed >> 32), 0u, 0u, 0u,
                 0u, 0u, 0u, counter, purpose, (u32)index, (u32)(index >> 32)};
    u32 x[16];
#pragma unroll
    for (int i = 0; i < 16; i++) x[i] = s[i];
#define QRD(a, b, c, d)                                                                                            \
    x[a] += x[b]; x[d] = rotl(x[d] ^ x[a], 16);                                                                    \
    x[c] += x[d]; x[b] = rotl(x[b] ^ x[c], 12);                                                                    \
    x[a] += x[b]; x[d] = rotl(x[d] ^ x[a], 8);                                                                     \
    x[c] += x[d]; x[b] = rotl(x[b] ^ x[c], 7);
#pragma unroll
    for (int i = 0; i < 10; i++) {
        QRD(0, 4, 8, 12) QRD(1, 5, 9, 13) QRD(2, 6, 10, 14) QRD(3, 7, 11, 15)
        QRD(0, 5, 10, 15) QRD(1, 6, 11, 12) QRD(2, 7, 8, 13) QRD(3, 4, 9, 14)
    }
#undef QRD
#pragma unroll
    for (int i = 0; i < 16; i++) out[i] = x[i] + s[i];
}

// x mod q for any 64-bit x, through two Montgomery reductions
DEV u64 mod64(u64 x, const PrimeC &pc) { return redc(0, mont_mul(x, pc.r2, pc.q, pc.qinv_neg), pc.q, pc.qinv_neg); }

// coefficient c = limb*n + t takes stream words 2c (high half) and 2c+1 (low half); one block = 4 coefficients
__global__ void k_sample_uniform(u64 *out, u64 seed, u32 purpose, u64 index, const u32 *pmap, u32 nlimbs,
                                 DevTables T)
{
    const u64 blk = (u64)blockIdx.x * EW_THREADS + threadIdx.x;
    const u64 total = (u64)nlimbs * T.n;
    if (blk * 4 >= total) return;
    u32 o[16];
    chacha_block(seed, purpose, index, (u32)blk, o);
#pragma unroll
    for (int i = 0; i < 4; i++) {
        u64 c = blk * 4 + i;
        if (c >= total) break;
        u64 hi = (u64)o[4 * i] | ((u64)o[4 * i + 1] << 32);
        u64 lo = (u64)o[4 * i + 2] | ((u64)o[4 * i + 3] << 32);
        u32 limb = (u32)(c >> T.logn);
        PrimeC pc = T.pc[pmap[limb]];
        // (hi * 2^64 + lo) mod q: with h = hi mod q the value h:lo < q 2^64, so
        // redc(h:lo) = value * 2^-64 and one more multiplication by 2^128 mod q
        // (Montgomery form of 2^64) restores it.
        u64 h = mod64(hi, pc);
        u64 v = redc(h, lo, pc.q, pc.qinv_neg);
        out[c] = mont_mul(v, pc.r2, pc.q, pc.qinv_neg);
    }
}
void hec_sample_uniform(const DevTables &T, u64 *out, u64 seed, u32 purpose, u64 index, const u32 *pmap,
                        int nlimbs, hipStream_t st)
{
    u64 blocks = ((u64)nlimbs * T.n + 3) / 4;
    dim3 g((blocks + EW_THREADS - 1) / EW_THREADS);
    hipLaunchKernelGGL(k_sample_uniform, g, dim3(EW_THREADS), 0, st, out, seed, purpose, index, pmap, (u32)nlimbs, T);
}

// kind 0: ternary, word w -> (w mod 3) - 1; kind 1: Gaussian by table inversion, bit 0 = sign
#define HEC_GAUSS_K 19
__global__ void k_sample_small(int64_t *out, u64 seed, u32 purpose, u64 index, int kind, const u64 *gT, DevTables T)
{
    const u64 blk = (u64)blockIdx.x * EW_THREADS + threadIdx.x;
    if (blk * 8 >= T.n) return;
    u32 o[16];
    chacha_block(seed, purpose, index, (u32)blk, o);
    for (int i = 0; i < 8; i++) {
        u64 t = blk * 8 + i;
        u64 w = (u64)o[2 * i] | ((u64)o[2 * i + 1] << 32);
        int64_t v;
        if (kind == 0) v = (int64_t)(w % 3) - 1;
        else {
            u64 r = w >> 1;
            int64_t mag = HEC_GAUSS_K;
            for (int j = 0; j < HEC_GAUSS_K; j++)
                if (r < gT[j]) { mag = j; break; }
            v = (w & 1) ? -mag : mag;
        }
        out[t] = v;
    }
}
void hec_sample_small(const DevTables &T, int64_t *out, u64 seed, u32 purpose, u64 index, int kind,
                      const u64 *gauss_T, hipStream_t st)
{
    u64 blocks = (T.n + 7) / 8;
    dim3 g((blocks + EW_THREADS - 1) / EW_THREADS);
    hipLaunchKernelGGL(k_sample_small, g, dim3(EW_THREADS), 0, st, out, seed, purpose, index, kind, gauss_T, T);
}

// ---------------------------------------------------------------------------
// fast base conversion (coefficient form)
// ---------------------------------------------------------------------------
// Workgroup (x, y, z): 256 coefficients; outputs y*per .. y*per+per-1 of
// descriptor dd[(z % group) * dstride], source src + (z / group)*sps,
// destination dst + z*dps (groups of `group` polynomials share a source, e.g.
// the digits of one ModUp).  Each lane computes its coefficient's a_i once and
// then every output of its group from them, so the inputs are read and scaled
// once per coefficient, not once per group of eight outputs; the descriptor's
// matrix and the output primes' constants are staged in LDS (every lane reads
// the same word: a broadcast).  NIN (the number of inputs) is a compile-time
// constant so that the a_i stay in registers.  With copy_in the lanes of the
// first output group also copy the inputs to the same positions of the
// destination (a ModUp digit then holds all its limbs).
#define BC_THREADS 256
template <int NIN>
__global__ void __launch_bounds__(BC_THREADS) k_bconv(const BconvDesc *dd, u32 dstride, u32 group, const u64 *src,
                                                      u64 *dst, size_t sps, size_t dps, u32 per, u32 copy_in,
                                                      DevTables T)
{
    __shared__ u64 hat[HEC_MAX_BCONV_IN * HEC_MAX_LIMBS];
    __shared__ u64 oq[HEC_MAX_LIMBS], oqi[HEC_MAX_LIMBS];
    __shared__ u32 opos[HEC_MAX_LIMBS];
    const BconvDesc *d = dd + (blockIdx.z % group) * dstride;
    const u32 nout = d->nout, nin = d->nin;
    const u32 j0 = blockIdx.y * per;
    const u32 j1 = j0 + per < nout ? j0 + per : nout;
    for (u32 e = threadIdx.x; e < NIN * nout; e += BC_THREADS) hat[e] = e < nin * nout ? split30(d->hat_m[e]) : 0;
    for (u32 j = threadIdx.x; j < nout; j += BC_THREADS) {
        const PrimeC pc = T.pc[d->out_prime[j]];
        oq[j] = pc.q;
        oqi[j] = pc.qinv_neg;
        opos[j] = d->out_pos[j];
    }
    __syncthreads();
    const size_t n = T.n;
    const u32 t = blockIdx.x * BC_THREADS + threadIdx.x;
    if (t >= n || j0 >= nout) return;
    const u64 *s = src + (blockIdx.z / group) * sps;
    u64 *o = dst + blockIdx.z * dps;
    // a_i in split form; rows past nin (a partial digit) are zero on both
    // sides, so their products vanish without a branch
    u64 a[NIN];
#pragma unroll
    for (int i = 0; i < NIN; i++) {
        a[i] = 0;
        if ((u32)i < nin) {
            const u64 x = s[(size_t)d->in_pos[i] * n + t];
            if (copy_in && blockIdx.y == 0) o[(size_t)d->in_pos[i] * n + t] = x;
            const u64 q = T.pc[d->in_prime[i]].q;
            a[i] = split30(shoup_mul(x, d->inv_hat[i], d->inv_hat_sh[i], q));
        }
    }
    for (u32 j = j0; j < j1; j++) {
        acc30 acc = {0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < NIN; i++) mac30(acc, a[i], hat[i * nout + j]);
        u64 lo, hi;
        acc30_total(acc, lo, hi);
        o[(size_t)opos[j] * n + t] = redc(hi, lo, oq[j], oqi[j]);
    }
}
template <int NIN>
static void bconv_launch(dim3 g, uint64_t units, hipStream_t st, const BconvDesc *d_desc, u32 dstride, u32 group,
                         const u64 *src, u64 *dst, size_t sps, size_t dps, u32 per, u32 copy_in, const DevTables &T)
{
    KLAUNCH("k_bconv", units, k_bconv<NIN>, g, dim3(BC_THREADS), 0, st, d_desc, dstride, group, src, dst, sps, dps,
            per, copy_in, T);
}
// nin_max: the largest input count among the launch's descriptors (the digits
// of a ModUp have alpha inputs but a partial last one)
void hec_bconv(const DevTables &T, const BconvDesc *d_desc, int desc_stride, int group, int nout_max, const u64 *src,
               u64 *dst, size_t src_poly_stride, size_t dst_poly_stride, int npolys, int copy_in, hipStream_t st,
               int nin_max)
{
    const int nin = nin_max;
    if (npolys <= 0 || group <= 0 || nin < 1 || nin > HEC_MAX_BCONV_IN) return;
    // all outputs of a coefficient in one lane when the launch has workgroups
    // enough to fill the chip; else groups of 8 outputs (more, smaller lanes)
    const u32 chunks = (T.n + BC_THREADS - 1) / BC_THREADS;
    const u32 per = (uint64_t)chunks * npolys >= 2048 ? (u32)nout_max : 8u;
    const u32 ngroups = ((u32)nout_max + per - 1) / per;
    dim3 g(chunks, ngroups, npolys);
#define BCV_ARGS g, (uint64_t)npolys, st, d_desc, (u32)desc_stride, (u32)group, src, dst, src_poly_stride, \
                 dst_poly_stride, per, (u32)(copy_in ? 1 : 0), T
    switch (nin) {
    case 1: bconv_launch<1>(BCV_ARGS); break;
    case 2: bconv_launch<2>(BCV_ARGS); break;
    case 3: bconv_launch<3>(BCV_ARGS); break;
    case 4: bconv_launch<4>(BCV_ARGS); break;
    case 5: bconv_launch<5>(BCV_ARGS); break;
    case 6: bconv_launch<6>(BCV_ARGS); break;
    case 7: bconv_launch<7>(BCV_ARGS); break;
    case 8: bconv_launch<8>(BCV_ARGS); break;
    case 9: bconv_launch<9>(BCV_ARGS); break;
    case 10: bconv_launch<10>(BCV_ARGS); break;
    case 11: bconv_launch<11>(BCV_ARGS); break;
    case 12: bconv_launch<12>(BCV_ARGS); break;
    case 13: bconv_launch<13>(BCV_ARGS); break;
    case 14: bconv_launch<14>(BCV_ARGS); break;
    case 15: bconv_launch<15>(BCV_ARGS); break;
    default: bconv_launch<16>(BCV_ARGS);
    }
#undef BCV_ARGS
}

// ---------------------------------------------------------------------------
// key-switch inner product with the automorphism folded into the read:
//   e_p[o][k] = sum_j D_j[o][perm_g(k)] * key_{g,j,p}[pmap[o]][k]
// ---------------------------------------------------------------------------
// Flat grid, XCD-aware: each XCD walks a contiguous run of (limb, rotation,
// chunk) items, so the hoisted digits of a limb are read from HBM once per
// XCD and reused from its L2 by every rotation of the batch.
__global__ void __launch_bounds__(EW_THREADS) k_ks_inner(KsBatch kb, const u64 *D, u32 beta, u32 nqp,
                                                         const u32 *pmap, u32 NLK, u32 nrot, u32 nchunks,
                                                         const u64 *pm, u32 nq, DevTables T)
{
    const u32 w = blockIdx.x, total = gridDim.x;
    const u32 i = (total & 7) ? w : (w & 7) * (total >> 3) + (w >> 3);
    const u32 chunk = i % nchunks, rest = i / nchunks;
    const u32 r = rest % nrot, o = rest / nrot;
    const u32 k = chunk * EW_THREADS + threadIdx.x;
    if (k >= T.n) return;
    const u32 pi = pmap[o];
    const PrimeC pc = T.pc[pi];
    const u32 src = auto_src(k, kb.g[r], T.logn);
    const size_t n = T.n;
    const u64 *key = kb.key[r];
    const u64 *Dr = kb.D[r] ? kb.D[r] : D;
    // the key is streamed once (non-temporal, so that it does not evict from
    // L2 the hoisted digits that every rotation of the launch reads again)
    acc128 a0 = {0, 0}, a1 = {0, 0};
    for (u32 j = 0; j < beta; j++) {
        u64 d = Dr[((size_t)j * nqp + o) * n + src];
        mac(a0, d, __builtin_nontemporal_load(key + (((size_t)j * 2 + 0) * NLK + pi) * n + k));
        mac(a1, d, __builtin_nontemporal_load(key + (((size_t)j * 2 + 1) * NLK + pi) * n + k));
    }
    // P * sigma_g(c0) on a Q limb of polynomial 0 (beta + 1 products below
    // q * 2^64): the ModDown's epilogue then reads no c0
    if (kb.c0[r] && o < nq) mac(a0, kb.c0[r][(size_t)o * n + src], pm[o]);
    // written past the caches too (read back by the ModDowns after the launch)
    u64 *out = kb.out[r];
    __builtin_nontemporal_store(redc(a0.hi, a0.lo, pc.q, pc.qinv_neg), out + (size_t)o * n + k);
    __builtin_nontemporal_store(redc(a1.hi, a1.lo, pc.q, pc.qinv_neg), out + ((size_t)nqp + o) * n + k);
}
void hec_ks_inner(const DevTables &T, const KsBatch &kb, int nrot, const u64 *D, int beta, int nqp, const u32 *pmap,
                  int NLK, hipStream_t st, const u64 *pm, int nq)
{
    const u32 nchunks = (T.n + EW_THREADS - 1) / EW_THREADS;
    dim3 g(nchunks * (u32)nqp * (u32)nrot);
    // units: limbs moved -- per rotation its 2 beta key limbs read and 2
    // products written per limb; the shared digits (beta limbs per limb, or
    // each entry's own) and the folded c0 limbs read once
    uint64_t units = 0, own = 0, fold = 0;
    for (int r = 0; r < nrot; r++) {
        own += kb.D[r] ? 1 : 0;
        fold += (pm && kb.c0[r]) ? 1 : 0;
    }
    units = (uint64_t)nrot * nqp * (2 * beta + 2) + (uint64_t)(D ? 1 + own : own) * beta * nqp +
            (fold ? (uint64_t)nq : 0);
    KLAUNCH("k_ks_inner", units, k_ks_inner, g, dim3(EW_THREADS), 0, st, kb, D, (u32)beta, (u32)nqp, pmap, (u32)NLK,
            (u32)nrot, nchunks, pm, (u32)(pm ? nq : 0), T);
}

// Key-stationary form of the same products for several inputs that share the
// rotations of a launch (the image shards of a layer): each thread loads its
// coefficient of the term's key limbs once into registers and loops over the
// inputs, so a key is read from HBM once per launch instead of once per input.
// Same accumulation as k_ks_inner (digits in order, one reduction), so the
// same residues.  Flat grid over (limb, rotation, chunk) in plain order:
// workgroups are dealt to the 8 XCDs round-robin, so all of them work on the
// same limb at a time and the digits of that limb for every input (beta limbs
// per input, 48 MiB for 32 inputs -- beyond one XCD's L2) are read from HBM
// once and by the other rotations of the launch from the shared last-level
// cache.  (k_ks_inner, whose limb's digits fit one L2, walks one contiguous
// run of items per XCD instead.)
template <int BETA>
__global__ void __launch_bounds__(EW_THREADS) k_ks_inner_multi(KsMulti kb, const u64 *D, size_t dstride, u32 S,
                                                               size_t estride, u32 beta_rt, u32 nqp, const u32 *pmap,
                                                               u32 NLK, u32 nrot, u32 nchunks, DevTables T)
{
    const u32 i = blockIdx.x;
    const u32 chunk = i % nchunks, rest = i / nchunks;
    const u32 r = rest % nrot, o = rest / nrot;
    const u32 k = chunk * EW_THREADS + threadIdx.x;
    if (k >= T.n) return;
    const u32 beta = BETA ? BETA : beta_rt;
    const u32 pi = pmap[o];
    const PrimeC pc = T.pc[pi];
    const u32 src = auto_src(k, kb.g[r], T.logn);
    const size_t n = T.n;
    const u64 *key = kb.key[r];
    const u64 m = kb.mask[r];
    u64 *out = kb.out[r];
    u64 kb0[BETA ? BETA : 1], kb1[BETA ? BETA : 1];
    if (BETA) {
#pragma unroll
        for (int j = 0; j < BETA; j++) {
            kb0[j] = __builtin_nontemporal_load(key + (((size_t)j * 2 + 0) * NLK + pi) * n + k);
            kb1[j] = __builtin_nontemporal_load(key + (((size_t)j * 2 + 1) * NLK + pi) * n + k);
        }
    }
    for (u32 u = 0; u < S; u++) {
        if (!((m >> u) & 1)) continue;
        const u64 *Du = D + (size_t)u * dstride;
        acc128 a0 = {0, 0}, a1 = {0, 0};
        if (BETA) {
#pragma unroll
            for (int j = 0; j < BETA; j++) {
                const u64 d = Du[((size_t)j * nqp + o) * n + src];
                mac(a0, d, kb0[j]);
                mac(a1, d, kb1[j]);
            }
        } else {
            for (u32 j = 0; j < beta; j++) {
                const u64 d = Du[((size_t)j * nqp + o) * n + src];
                mac(a0, d, key[(((size_t)j * 2 + 0) * NLK + pi) * n + k]);
                mac(a1, d, key[(((size_t)j * 2 + 1) * NLK + pi) * n + k]);
            }
        }
        // written past the caches: 2 limbs per input and rotation, read back
        // only by the ModDowns after the launch
        u64 *e = out + (size_t)u * estride;
        __builtin_nontemporal_store(redc(a0.hi, a0.lo, pc.q, pc.qinv_neg), e + (size_t)o * n + k);
        __builtin_nontemporal_store(redc(a1.hi, a1.lo, pc.q, pc.qinv_neg), e + ((size_t)nqp + o) * n + k);
    }
}
template <int BETA>
static void ks_inner_multi_launch(dim3 g, uint64_t units, hipStream_t st, const KsMulti &kb, const u64 *D,
                                  size_t dstride, u32 S, size_t estride, u32 beta, u32 nqp, const u32 *pmap, u32 NLK,
                                  u32 nrot, u32 nchunks, const DevTables &T)
{
    KLAUNCH("k_ks_inner_multi", units, k_ks_inner_multi<BETA>, g, dim3(EW_THREADS), 0, st, kb, D, dstride, S, estride,
            beta, nqp, pmap, NLK, nrot, nchunks, T);
}
bool hec_ks_inner_multi(const DevTables &T, const KsMulti &kb, int nrot, const u64 *D, size_t dstride, int S,
                        size_t estride, int beta, int nqp, const u32 *pmap, int NLK, hipStream_t st)
{
    if (nrot < 1 || nrot > HEC_KS_BATCH || S < 1 || S > HEC_MULTI_MAX_INPUTS || beta < 1) return false;
    const u32 nchunks = (T.n + EW_THREADS - 1) / EW_THREADS;
    dim3 g(nchunks * (u32)nqp * (u32)nrot);
    // units: key limbs read once, digits once per input, outputs written
    const uint64_t units = (uint64_t)nrot * 2 * beta * nqp + (uint64_t)S * beta * nqp + (uint64_t)nrot * S * 2 * nqp;
#define KSM_ARGS g, units, st, kb, D, dstride, (u32)S, estride, (u32)beta, (u32)nqp, pmap, (u32)NLK, (u32)nrot, nchunks, T
    switch (beta) {
    case 1: ks_inner_multi_launch<1>(KSM_ARGS); break;
    case 2: ks_inner_multi_launch<2>(KSM_ARGS); break;
    case 3: ks_inner_multi_launch<3>(KSM_ARGS); break;
    case 4: ks_inner_multi_launch<4>(KSM_ARGS); break;
    default: ks_inner_multi_launch<0>(KSM_ARGS);
    }
#undef KSM_ARGS
    return true;
}

// Key switching fused with the plaintext products of a convolution, summed
// before ModDown (one ModDown per output instead of one per rotation).  The
// term sigma_g(c0) of a rotation is folded in as P * sigma_g(c0) on the Q limbs:
// ModDown(E + P*A) = ModDown(E) + A exactly.  Products are summed into 128 bits
// and reduced once: < (beta + 1) q^2 for the key switch and < HEC_KS_BATCH q^2
// for the terms, both below q * 2^64 (checked at context creation).
//
// Each lane takes two adjacent coefficients k, k+1 (k even) so that every
// access is a 16-byte load: the automorphism maps the pair onto the pair
// {src, src ^ 1} (k and k+1 differ in the top bit of brv(k), i.e. by n in the
// exponent 2 brv(k) + 1, which g odd keeps at n: the source index flips its
// lowest bit).  BETA and NOUT are compile-time so that all loads of a term
// are issued together; terms [0, nz) are rotations by zero, the rest are not.
typedef u64 u64x2 __attribute__((ext_vector_type(2)));
DEV u64x2 ld2(const u64 *p) { return *(const u64x2 *)p; }
// streamed once (keys, plaintexts): non-temporal, so that they do not evict the
// hoisted digits that every rotation of the launch re-reads from L2
DEV u64x2 ld2_stream(const u64 *p) { return __builtin_nontemporal_load((const u64x2 *)p); }
DEV void st2(u64 *p, u64x2 v) { *(u64x2 *)p = v; }

// one output per workgroup with plaintexts as given: at most 96 registers,
// five waves per SIMD (the kernel is bound by its key stream and needs the
// waves to cover latency)
template <int BETA, int NOUT>
__global__ void __launch_bounds__(EW_THREADS) __attribute__((amdgpu_waves_per_eu(NOUT == 1 ? 5 : 4)))
k_ks_mac(KsMacBatch b, u32 nz, u32 nterms, u32 beta_rt, u32 nq, u32 nqp, const u32 *pmap, const u64 *pm, u32 NLK,
         u32 first, u32 nchunks, u32 ngroups, ShardArg sh, DevTables T)
{
    const u32 w = blockIdx.x, total = gridDim.x;
    const u32 i0 = (total & 7) ? w : (w & 7) * (total >> 3) + (w >> 3);
    // the inputs of a multi-input launch (same terms, keys and plaintexts) are
    // the fastest index, then the output groups: the workgroups of one (limb,
    // chunk) are neighbours, run together on one XCD and share the key,
    // plaintext and digit reads through its L2
    const u32 u = i0 % sh.S, i = i0 / sh.S;
    const u32 grp = i % ngroups, rest = i / ngroups;
    const u32 chunk = rest % nchunks, o = rest / nchunks;
    const u32 vb = grp * NOUT;
    const u32 k = 2 * (chunk * EW_THREADS + threadIdx.x);
    if (k >= T.n) return;
    const u32 beta = BETA ? BETA : beta_rt;
    const size_t n = T.n;
    const u32 pi = pmap[o];
    const PrimeC pc = T.pc[pi];
    const bool isq = o < nq;
    const u64 pmo = isq ? pm[o] : 0;
    acc128 acc[NOUT][2][2];  // [output][poly][coefficient]
#pragma unroll
    for (int v = 0; v < NOUT; v++)
#pragma unroll
        for (int p = 0; p < 2; p++) acc[v][p][0] = acc[v][p][1] = acc128{0, 0};
    // rotations by zero: P * (c0, c1)
    if (isq)
        for (u32 t = 0; t < nz; t++) {
            const u64 *ct = b.ct[t] + u * sh.cs;
            const u64x2 c0 = ld2(ct + (size_t)o * n + k), c1 = ld2(ct + ((size_t)nq + o) * n + k);
            const u64 e00 = mont_mul(c0.x, pmo, pc.q, pc.qinv_neg), e01 = mont_mul(c0.y, pmo, pc.q, pc.qinv_neg);
            const u64 e10 = mont_mul(c1.x, pmo, pc.q, pc.qinv_neg), e11 = mont_mul(c1.y, pmo, pc.q, pc.qinv_neg);
#pragma unroll
            for (int v = 0; v < NOUT; v++) {
                const u64 *pt = b.pt[t][vb + v];
                if (!pt) continue;
                const u64x2 m = ld2(pt + (size_t)o * n + k);
                mac(acc[v][0][0], e00, m.x);
                mac(acc[v][0][1], e01, m.y);
                mac(acc[v][1][0], e10, m.x);
                mac(acc[v][1][1], e11, m.y);
            }
        }
    for (u32 t = nz; t < nterms; t++) {
        const u32 src = auto_src(k, b.g[t], T.logn);
        const u32 sb = src & ~1u;
        const bool sw = src & 1u;
        const u64 *key = b.key[t], *D = b.D[t] + u * sh.ds, *ct = b.ct[t] + u * sh.cs;
        // issue the loads of the input and plaintext limbs together with the key
        // loads below (addresses always valid; unused values are ignored)
        const u64x2 c = ld2(ct + (size_t)(isq ? o : 0) * n + sb);
        u64x2 m[NOUT];
#pragma unroll
        for (int v = 0; v < NOUT; v++) {
            const u64 *pt = b.pt[t][vb + v];
            m[v] = ld2_stream((pt ? pt : ct) + (size_t)(pt ? o : 0) * n + k);
        }
        acc128 a00 = {0, 0}, a01 = {0, 0}, a10 = {0, 0}, a11 = {0, 0};  // [poly][coefficient]
#pragma unroll
        for (u32 j = 0; j < beta; j++) {
            const u64x2 d = ld2(D + ((size_t)j * nqp + o) * n + sb);
            const u64x2 kb = ld2_stream(key + (((size_t)j * 2 + 0) * NLK + pi) * n + k);
            const u64x2 ka = ld2_stream(key + (((size_t)j * 2 + 1) * NLK + pi) * n + k);
            const u64 d0 = sw ? d.y : d.x, d1 = sw ? d.x : d.y;
            mac(a00, d0, kb.x);
            mac(a01, d1, kb.y);
            mac(a10, d0, ka.x);
            mac(a11, d1, ka.y);
        }
        if (isq) {
            mac(a00, sw ? c.y : c.x, pmo);
            mac(a01, sw ? c.x : c.y, pmo);
        }
        const u64 e00 = redc(a00.hi, a00.lo, pc.q, pc.qinv_neg), e01 = redc(a01.hi, a01.lo, pc.q, pc.qinv_neg);
        const u64 e10 = redc(a10.hi, a10.lo, pc.q, pc.qinv_neg), e11 = redc(a11.hi, a11.lo, pc.q, pc.qinv_neg);
#pragma unroll
        for (int v = 0; v < NOUT; v++) {
            if (!b.pt[t][vb + v]) continue;
            mac(acc[v][0][0], e00, m[v].x);
            mac(acc[v][0][1], e01, m[v].y);
            mac(acc[v][1][0], e10, m[v].x);
            mac(acc[v][1][1], e11, m[v].y);
        }
    }
#pragma unroll
    for (int v = 0; v < NOUT; v++) {
        u64 *E = b.E[vb + v];
        if (!E) continue;
        E += u * sh.es;
#pragma unroll
        for (int p = 0; p < 2; p++) {
            u64 *dst = E + ((size_t)p * nqp + o) * n + k;
            u64x2 r;
            r.x = redc(acc[v][p][0].hi, acc[v][p][0].lo, pc.q, pc.qinv_neg);
            r.y = redc(acc[v][p][1].hi, acc[v][p][1].lo, pc.q, pc.qinv_neg);
            if (!((first >> (vb + v)) & 1)) {
                const u64x2 old = ld2(dst);
                r.x = add_mod(r.x, old.x, pc.q);
                r.y = add_mod(r.y, old.y, pc.q);
            }
            st2(dst, r);
        }
    }
}

// The same for many outputs: one coefficient per lane and up to KSW_OUT
// outputs per workgroup (`per` of them used), so that the key-switch product
// of a term is computed once for that many outputs; output groups of the same
// (limb, chunk) are neighbours and share the key and digit reads through L2.
#define KSW_OUT 8
template <int BETA>
__global__ void __launch_bounds__(EW_THREADS) k_ks_mac_w(KsMacBatch b, u32 nz, u32 nterms, u32 beta_rt, u32 nq,
                                                         u32 nqp, const u32 *pmap, const u64 *pm, u32 NLK,
                                                         u32 first, u32 nchunks, u32 ngroups, u32 per, u32 nout,
                                                         DevTables T)
{
    const u32 w = blockIdx.x, total = gridDim.x;
    const u32 i = (total & 7) ? w : (w & 7) * (total >> 3) + (w >> 3);
    const u32 grp = i % ngroups, rest = i / ngroups;
    const u32 chunk = rest % nchunks, o = rest / nchunks;
    const u32 vb = grp * per;
    const u32 k = chunk * EW_THREADS + threadIdx.x;
    if (k >= T.n) return;
    const u32 beta = BETA ? BETA : beta_rt;
    const size_t n = T.n;
    const u32 pi = pmap[o];
    const PrimeC pc = T.pc[pi];
    const bool isq = o < nq;
    const u64 pmo = isq ? pm[o] : 0;
    const u32 nv = vb + per <= nout ? per : (vb < nout ? nout - vb : 0);
    acc128 acc[KSW_OUT][2];
#pragma unroll
    for (int v = 0; v < KSW_OUT; v++) acc[v][0] = acc[v][1] = acc128{0, 0};
    if (isq)
        for (u32 t = 0; t < nz; t++) {
            const u64 *ct = b.ct[t];
            const u64 e0 = mont_mul(ct[(size_t)o * n + k], pmo, pc.q, pc.qinv_neg);
            const u64 e1 = mont_mul(ct[((size_t)nq + o) * n + k], pmo, pc.q, pc.qinv_neg);
#pragma unroll
            for (u32 v = 0; v < KSW_OUT; v++) {
                if (v >= nv) break;
                const u64 *pt = b.pt[t][vb + v];
                if (!pt) continue;
                const u64 m = pt[(size_t)o * n + k];
                mac(acc[v][0], e0, m);
                mac(acc[v][1], e1, m);
            }
        }
    for (u32 t = nz; t < nterms; t++) {
        const u32 src = auto_src(k, b.g[t], T.logn);
        const u64 *key = b.key[t], *D = b.D[t], *ct = b.ct[t];
        const u64 c = ct[(size_t)(isq ? o : 0) * n + src];
        u64 m[KSW_OUT];
#pragma unroll
        for (u32 v = 0; v < KSW_OUT; v++) {
            const u64 *pt = v < nv ? b.pt[t][vb + v] : nullptr;
            m[v] = pt ? __builtin_nontemporal_load(pt + (size_t)o * n + k) : 0;
        }
        acc128 a0 = {0, 0}, a1 = {0, 0};
#pragma unroll
        for (u32 j = 0; j < beta; j++) {
            const u64 d = D[((size_t)j * nqp + o) * n + src];
            mac(a0, d, key[(((size_t)j * 2 + 0) * NLK + pi) * n + k]);
            mac(a1, d, key[(((size_t)j * 2 + 1) * NLK + pi) * n + k]);
        }
        if (isq) mac(a0, c, pmo);
        const u64 e0 = redc(a0.hi, a0.lo, pc.q, pc.qinv_neg), e1 = redc(a1.hi, a1.lo, pc.q, pc.qinv_neg);
#pragma unroll
        for (u32 v = 0; v < KSW_OUT; v++) {
            if (v >= nv) break;
            if (!b.pt[t][vb + v]) continue;
            mac(acc[v][0], e0, m[v]);
            mac(acc[v][1], e1, m[v]);
        }
    }
#pragma unroll
    for (u32 v = 0; v < KSW_OUT; v++) {
        if (v >= nv) break;
        u64 *E = b.E[vb + v];
        if (!E) continue;
#pragma unroll
        for (int p = 0; p < 2; p++) {
            u64 *dst = E + ((size_t)p * nqp + o) * n + k;
            u64 r = redc(acc[v][p].hi, acc[v][p].lo, pc.q, pc.qinv_neg);
            if (!((first >> (vb + v)) & 1)) r = add_mod(r, *dst, pc.q);
            *dst = r;
        }
    }
}

// Basis-mask plaintexts (BasisArg): for term t the basis polynomials E_b are
// read once and y_{b,p} = x_p * E_b mod q formed for all outputs of the
// workgroup (x the key-switch output, or P * c for a rotation by zero); output
// v then adds sum_b w_{t,v,b} y_{b,p} with the weights small signed integers
// (|w| < 2^31, checked when the plan is built): 64 x 32-bit products summed
// exactly in 128-bit two's complement (|sum| < 64 * 2^91 = 2^97 for at most 16
// terms of 4 blocks), reduced once with the offset q * 2^62 (>= 2^97 for
// q >= 2^35, so the sum is non-negative and below q * 2^64), which is
// congruent to 0.  The residues equal (sum_b w_b E_b) * x mod q exactly.
DEV void smac(acc128 &acc, u64 y, int64_t w)
{
    const u32 a = (u32)(w < 0 ? -w : w);
    const u64 p0 = (u64)(u32)y * a;
    const u64 p1 = (u64)(u32)(y >> 32) * a + (p0 >> 32);
    const u64 lo = (u64)(u32)p0 | (p1 << 32), hi = p1 >> 32;
    if (w >= 0) {
        acc.lo += lo;
        acc.hi += hi + (acc.lo < lo ? 1 : 0);
    } else {
        const u64 borrow = acc.lo < lo ? 1 : 0;
        acc.lo -= lo;
        acc.hi -= hi + borrow;
    }
}
// acc mod q in [0, q): redc of acc + q 2^62 is acc * 2^-64, times (2^64)^2 mod q in Montgomery form
DEV u64 sfinal(acc128 acc, const PrimeC &pc)
{
    const u64 klo = pc.q << 62, khi = pc.q >> 2;
    acc.lo += klo;
    acc.hi += khi + (acc.lo < klo ? 1 : 0);
    return mont_mul(redc(acc.hi, acc.lo, pc.q, pc.qinv_neg), pc.r2, pc.q, pc.qinv_neg);
}
DEV void basis_y(const BasisArg &ba, u32 t, u32 o, u32 k, size_t n, u64 x0, u64 x1, const PrimeC &pc,
                 u64 (&y)[HEC_BASIS_NB][2])
{
    const u64 *Et = ba.E + ((size_t)ba.tap[t] * ba.nb * ba.nqp + o) * n + k;
#pragma unroll
    for (u32 b = 0; b < HEC_BASIS_NB; b++) {
        const u64 e = b < ba.nb ? Et[(size_t)b * ba.nqp * n] : 0;
        y[b][0] = mont_mul(x0, e, pc.q, pc.qinv_neg);
        y[b][1] = mont_mul(x1, e, pc.q, pc.qinv_neg);
    }
}
DEV void basis_add(acc128 (&acc)[2], const int64_t *W, const BasisArg &ba, const u64 (&y)[HEC_BASIS_NB][2])
{
#pragma unroll
    for (u32 b = 0; b < HEC_BASIS_NB; b++)
        if (b < ba.nb) {
            smac(acc[0], y[b][0], W[b]);
            smac(acc[1], y[b][1], W[b]);
        }
}

// Key switching fused with basis-mask plaintext products: the layout of
// k_ks_mac_w (one coefficient per lane, up to KSW_OUT outputs per workgroup);
// pt[t][v] points at the nb signed weights of (term t, output v).
template <int BETA>
__global__ void __launch_bounds__(EW_THREADS) k_ks_mac_basis(KsMacBatch b, BasisArg ba, u32 nz, u32 nterms,
                                                             u32 beta_rt, u32 nq, u32 nqp, const u32 *pmap,
                                                             const u64 *pm, u32 NLK, u32 first, u32 nchunks,
                                                             u32 ngroups, u32 per, u32 nout, DevTables T)
{
    const u32 w = blockIdx.x, total = gridDim.x;
    const u32 i = (total & 7) ? w : (w & 7) * (total >> 3) + (w >> 3);
    const u32 grp = i % ngroups, rest = i / ngroups;
    const u32 chunk = rest % nchunks, o = rest / nchunks;
    const u32 vb = grp * per;
    const u32 k = chunk * EW_THREADS + threadIdx.x;
    if (k >= T.n) return;
    const u32 beta = BETA ? BETA : beta_rt;
    const size_t n = T.n;
    const u32 pi = pmap[o];
    const PrimeC pc = T.pc[pi];
    const bool isq = o < nq;
    const u64 pmo = isq ? pm[o] : 0;
    const u32 nv = vb + per <= nout ? per : (vb < nout ? nout - vb : 0);
    acc128 acc[KSW_OUT][2];
#pragma unroll
    for (int v = 0; v < KSW_OUT; v++) acc[v][0] = acc[v][1] = acc128{0, 0};
    for (u32 t = 0; t < nterms; t++) {
        const u64 *ct = b.ct[t];
        u64 x0, x1;
        if (t < nz) {
            // rotation by zero: P * (c0, c1) on the Q limbs, nothing on the P limbs
            if (!isq) continue;
            x0 = mont_mul(ct[(size_t)o * n + k], pmo, pc.q, pc.qinv_neg);
            x1 = mont_mul(ct[((size_t)nq + o) * n + k], pmo, pc.q, pc.qinv_neg);
        } else {
            const u32 src = auto_src(k, b.g[t], T.logn);
            const u64 *key = b.key[t], *D = b.D[t];
            const u64 c = ct[(size_t)(isq ? o : 0) * n + src];
            acc128 a0 = {0, 0}, a1 = {0, 0};
#pragma unroll
            for (u32 j = 0; j < beta; j++) {
                const u64 d = D[((size_t)j * nqp + o) * n + src];
                mac(a0, d, __builtin_nontemporal_load(key + (((size_t)j * 2 + 0) * NLK + pi) * n + k));
                mac(a1, d, __builtin_nontemporal_load(key + (((size_t)j * 2 + 1) * NLK + pi) * n + k));
            }
            if (isq) mac(a0, c, pmo);
            x0 = redc(a0.hi, a0.lo, pc.q, pc.qinv_neg);
            x1 = redc(a1.hi, a1.lo, pc.q, pc.qinv_neg);
        }
        u64 y[HEC_BASIS_NB][2];
        basis_y(ba, t, o, k, n, x0, x1, pc, y);
#pragma unroll
        for (u32 v = 0; v < KSW_OUT; v++) {
            if (v >= nv) break;
            const int64_t *W = (const int64_t *)b.pt[t][vb + v];
            if (W) basis_add(acc[v], W, ba, y);
        }
    }
#pragma unroll
    for (u32 v = 0; v < KSW_OUT; v++) {
        if (v >= nv) break;
        u64 *E = b.E[vb + v];
        if (!E) continue;
#pragma unroll
        for (int p = 0; p < 2; p++) {
            u64 *dst = E + ((size_t)p * nqp + o) * n + k;
            u64 r = sfinal(acc[v][p], pc);
            if (!((first >> (vb + v)) & 1)) r = add_mod(r, *dst, pc.q);
            *dst = r;
        }
    }
}

template <int BETA>
static void ks_mac_w_launch(dim3 g, uint64_t units, hipStream_t st, const KsMacBatch &b, const BasisArg *ba, u32 nz,
                            u32 nterms, u32 beta, u32 nq, u32 nqp, const u32 *pmap, const u64 *pm, u32 NLK,
                            u32 first, u32 nchunks, u32 ngroups, u32 per, u32 nout, const DevTables &T)
{
    if (ba)
        KLAUNCH("k_ks_mac", units, (k_ks_mac_basis<BETA>), g, dim3(EW_THREADS), 0, st, b, *ba, nz, nterms, beta, nq,
                nqp, pmap, pm, NLK, first, nchunks, ngroups, per, nout, T);
    else
        KLAUNCH("k_ks_mac", units, (k_ks_mac_w<BETA>), g, dim3(EW_THREADS), 0, st, b, nz, nterms, beta, nq, nqp,
                pmap, pm, NLK, first, nchunks, ngroups, per, nout, T);
}

template <int BETA, int NOUT>
static void ks_mac_launch(dim3 g, uint64_t units, hipStream_t st, const KsMacBatch &b, u32 nz, u32 nterms, u32 beta,
                          u32 nq, u32 nqp, const u32 *pmap, const u64 *pm, u32 NLK, u32 first, u32 nchunks,
                          u32 ngroups, const ShardArg &sh, const DevTables &T)
{
    KLAUNCH("k_ks_mac", units, (k_ks_mac<BETA, NOUT>), g, dim3(EW_THREADS), 0, st, b, nz, nterms, beta, nq, nqp,
            pmap, pm, NLK, first, nchunks, ngroups, sh, T);
}
template <int NOUT>
static void ks_mac_beta(dim3 g, uint64_t units, hipStream_t st, const KsMacBatch &b, u32 nz, u32 nterms, u32 beta,
                        u32 nq, u32 nqp, const u32 *pmap, const u64 *pm, u32 NLK, u32 first, u32 nchunks,
                        u32 ngroups, const DevTables &T, const ShardArg &sh = ShardArg{1, 0, 0, 0})
{
#define KSM_ARGS g, units, st, b, nz, nterms, beta, nq, nqp, pmap, pm, NLK, first, nchunks, ngroups, sh, T
    switch (beta) {
    case 1: ks_mac_launch<1, NOUT>(KSM_ARGS); break;
    case 2: ks_mac_launch<2, NOUT>(KSM_ARGS); break;
    case 3: ks_mac_launch<3, NOUT>(KSM_ARGS); break;
    case 4: ks_mac_launch<4, NOUT>(KSM_ARGS); break;
    default: ks_mac_launch<0, NOUT>(KSM_ARGS);
    }
#undef KSM_ARGS
}
// Work unit of the profiler: one limb (n words) moved to or from HBM, counting
// each key, plaintext and accumulator limb once and the hoisted digits and
// the input ciphertext of each distinct input once per launch (the output
// groups re-read them from L2).
bool hec_ks_mac(const DevTables &T, const KsMacBatch &b, int nterms, int nout, int beta, int nq, int nqp,
                const u32 *pmap, const u64 *pm, int NLK, int first, hipStream_t st, const BasisArg *ba)
{
    if (nterms < 0 || nterms > HEC_KS_BATCH || nout < 1 || nout > HEC_MAC_OUT) return false;
    if (ba && (!ba->E || ba->nb < 1 || ba->nb > HEC_BASIS_NB || (int)ba->nqp != nqp)) return false;
    u32 nz = 0;
    while ((int)nz < nterms && b.g[nz] == 1) nz++;
    for (int t = 0; t < nterms; t++) {
        if (!b.ct[t]) return false;
        if (t >= (int)nz && (b.g[t] == 1 || !b.key[t] || !b.D[t])) return false;  // zero rotations come first
    }
    uint64_t units = 0;
    for (int t = 0; t < nterms; t++) {
        bool new_ct = true, new_d = t >= (int)nz;
        for (int s = 0; s < t; s++) {
            if (b.ct[s] == b.ct[t]) new_ct = false;
            if (s >= (int)nz && b.D[s] == b.D[t]) new_d = false;
        }
        if (new_ct) units += (uint64_t)nq * (t < (int)nz ? 2 : 1);
        if (new_d) units += (uint64_t)beta * nqp;
        if (t >= (int)nz) units += 2ull * beta * nqp;
        if (ba) {
            bool new_tap = true;
            for (int s = 0; s < t; s++) new_tap &= ba->tap[s] != ba->tap[t];
            if (new_tap) units += (uint64_t)ba->nb * (t >= (int)nz ? nqp : nq);
        } else {
            for (int v = 0; v < nout; v++)
                if (b.pt[t][v]) units += t >= (int)nz ? nqp : nq;
        }
    }
    for (int v = 0; v < nout; v++) units += ((first >> v) & 1) ? 2ull * nqp : 4ull * nqp;
    KsMacBatch bb = b;
    for (int v = nout; v < HEC_MAC_OUT; v++) {
        bb.E[v] = nullptr;
        for (int t = 0; t < HEC_KS_BATCH; t++) bb.pt[t][v] = nullptr;
    }
    if (nout > 2 || ba) {
        // many outputs (or basis-mask plaintexts): one coefficient per lane, groups of at most KSW_OUT
        // outputs of even size
        const u32 ng = ((u32)nout + KSW_OUT - 1) / KSW_OUT, per = ((u32)nout + ng - 1) / ng;
        const u32 nch = (T.n + EW_THREADS - 1) / EW_THREADS;
        dim3 g(nch * (u32)nqp * ng);
#define KSW_ARGS g, units, st, bb, ba, nz, (u32)nterms, (u32)beta, (u32)nq, (u32)nqp, pmap, pm, (u32)NLK, (u32)first, \
                 nch, ng, per, (u32)nout, T
        switch (beta) {
        case 1: ks_mac_w_launch<1>(KSW_ARGS); break;
        case 2: ks_mac_w_launch<2>(KSW_ARGS); break;
        case 3: ks_mac_w_launch<3>(KSW_ARGS); break;
        case 4: ks_mac_w_launch<4>(KSW_ARGS); break;
        default: ks_mac_w_launch<0>(KSW_ARGS);
        }
#undef KSW_ARGS
        return true;
    }
    const u32 nchunks = (T.n / 2 + EW_THREADS - 1) / EW_THREADS;
    // outputs per workgroup: 1 or 2, two coefficients per lane
    const u32 per = (u32)nout;
    const u32 ngroups = 1;
    dim3 g(nchunks * (u32)nqp * ngroups);
    if (per == 1)
        ks_mac_beta<1>(g, units, st, bb, nz, nterms, beta, nq, nqp, pmap, pm, NLK, first, nchunks, ngroups, T);
    else
        ks_mac_beta<2>(g, units, st, bb, nz, nterms, beta, nq, nqp, pmap, pm, NLK, first, nchunks, ngroups, T);
    return true;
}

bool hec_ks_mac_shards(const DevTables &T, const KsMacBatch &b, int nterms, int beta, int nq, int nqp,
                       const u32 *pmap, const u64 *pm, int NLK, int first, const ShardArg &sh, hipStream_t st)
{
    if (nterms < 0 || nterms > HEC_KS_BATCH || sh.S < 1 || !b.E[0]) return false;
    u32 nz = 0;
    while ((int)nz < nterms && b.g[nz] == 1) nz++;
    for (int t = 0; t < nterms; t++) {
        if (!b.ct[t] || !b.pt[t][0]) return false;
        if (t >= (int)nz && (b.g[t] == 1 || !b.key[t] || !b.D[t])) return false;  // zero rotations come first
    }
    // units: every key and plaintext limb once, the inputs' digits and ciphertexts once, the accumulators
    uint64_t units = (uint64_t)sh.S * ((uint64_t)beta * nqp + 2ull * nq) + (((first & 1) ? 2ull : 4ull) * nqp) * sh.S;
    for (int t = 0; t < nterms; t++) units += (t >= (int)nz ? 2ull * beta * nqp : 0) + (t >= (int)nz ? nqp : nq);
    KsMacBatch bb = b;
    for (int v = 1; v < HEC_MAC_OUT; v++) {
        bb.E[v] = nullptr;
        for (int t = 0; t < HEC_KS_BATCH; t++) bb.pt[t][v] = nullptr;
    }
    const u32 nchunks = (T.n / 2 + EW_THREADS - 1) / EW_THREADS;
    dim3 g(nchunks * (u32)nqp * sh.S);
    ks_mac_beta<1>(g, units, st, bb, nz, (u32)nterms, (u32)beta, (u32)nq, (u32)nqp, pmap, pm, (u32)NLK, (u32)first,
                   nchunks, 1, T, sh);
    return true;
}

// Sums of plaintext products over Q: each lane one coefficient of one limb, the
// products of all terms for up to HEC_MAC_OUTS outputs accumulated in 128 bits
// (< HEC_MAC_TERMS q^2 < q 2^64) and reduced once, so every rotated input is
// read once per group of outputs.
// NOUT: outputs the accumulators are sized for (>= nout).  Up to four
// outputs the products are summed by 30-bit halves (acc30: four
// multiply-adds and no carry per product); eight keep the 128-bit form, whose
// accumulators take half the registers.  Same integer sums, same residues.
template <int NOUT>
__global__ void __launch_bounds__(EW_THREADS) k_mac_terms(MacBatch b, u32 nterms, u32 nout, u32 nq, u32 first,
                                                          DevTables T)
{
    constexpr bool SPLIT = NOUT <= 4;
    // limbs from the top: the reverse of the order in which the ModDown row
    // pass writes them, so the last written are read first
    const u32 o = gridDim.y - 1 - blockIdx.y;
    const size_t k = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= T.n) return;
    const PrimeC pc = T.pc[o];
    const size_t n = T.n, off = (size_t)o * n + k;
    acc30 s[SPLIT ? NOUT : 1][2];
    acc128 acc[SPLIT ? 1 : NOUT][2];
#pragma unroll
    for (int v = 0; v < (SPLIT ? NOUT : 1); v++) s[v][0] = s[v][1] = acc30{0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < (SPLIT ? 1 : NOUT); v++) acc[v][0] = acc[v][1] = acc128{0, 0};
    for (u32 t = 0; t < nterms; t++) {
        const u64 *ct = b.ct[t];
        const u64 c0 = ct[off], c1 = ct[(size_t)nq * n + off];
        const u64 c0s = split30(c0), c1s = split30(c1);
#pragma unroll
        for (int v = 0; v < NOUT; v++) {
            const u64 *pt = b.pt[t][v];
            if (!pt) continue;
            const u64 m = pt[off];
            if (SPLIT) {
                const u64 ms = split30(m);
                mac30(s[SPLIT ? v : 0][0], c0s, ms);
                mac30(s[SPLIT ? v : 0][1], c1s, ms);
            } else {
                mac(acc[SPLIT ? 0 : v][0], c0, m);
                mac(acc[SPLIT ? 0 : v][1], c1, m);
            }
        }
    }
#pragma unroll
    for (int v = 0; v < NOUT; v++) {
        u64 *out = b.out[v];
        if ((u32)v >= nout || !out) continue;
#pragma unroll
        for (int p = 0; p < 2; p++) {
            u64 *dst = out + (size_t)p * nq * n + off;
            u64 lo, hi;
            if (SPLIT) {
                acc30_total(s[SPLIT ? v : 0][p], lo, hi);
            } else {
                lo = acc[SPLIT ? 0 : v][p].lo;
                hi = acc[SPLIT ? 0 : v][p].hi;
            }
            u64 r = redc(hi, lo, pc.q, pc.qinv_neg);
            if (!((first >> v) & 1)) r = add_mod(r, *dst, pc.q);
            *dst = r;
        }
    }
}
template <int NOUT>
static void mac_terms_launch(dim3 g, hipStream_t st, const MacBatch &b, int nterms, int nout, int nq, int first,
                             const DevTables &T)
{
    KLAUNCH("k_mac_terms", (uint64_t)nq * nterms, k_mac_terms<NOUT>, g, dim3(EW_THREADS), 0, st, b, (u32)nterms,
            (u32)nout, (u32)nq, (u32)first, T);
}
// the same with basis-mask plaintexts: pt[t][v] points at the nb signed weights of (term t, output v)
__global__ void __launch_bounds__(EW_THREADS) k_mac_terms_basis(MacBatch b, BasisArg ba, u32 nterms, u32 nout, u32 nq,
                                                                u32 first, DevTables T)
{
    const u32 o = blockIdx.y;
    const u32 k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= T.n) return;
    const PrimeC pc = T.pc[o];
    const size_t n = T.n, off = (size_t)o * n + k;
    acc128 acc[HEC_MAC_OUTS][2];
#pragma unroll
    for (int v = 0; v < HEC_MAC_OUTS; v++) acc[v][0] = acc[v][1] = acc128{0, 0};
    for (u32 t = 0; t < nterms; t++) {
        const u64 *ct = b.ct[t];
        u64 y[HEC_BASIS_NB][2];
        basis_y(ba, t, o, k, n, ct[off], ct[(size_t)nq * n + off], pc, y);
#pragma unroll
        for (int v = 0; v < HEC_MAC_OUTS; v++) {
            const int64_t *W = (const int64_t *)b.pt[t][v];
            if (W) basis_add(acc[v], W, ba, y);
        }
    }
#pragma unroll
    for (int v = 0; v < HEC_MAC_OUTS; v++) {
        u64 *out = b.out[v];
        if ((u32)v >= nout || !out) continue;
#pragma unroll
        for (int p = 0; p < 2; p++) {
            u64 *dst = out + (size_t)p * nq * n + off;
            u64 r = sfinal(acc[v][p], pc);
            if (!((first >> v) & 1)) r = add_mod(r, *dst, pc.q);
            *dst = r;
        }
    }
}
bool hec_mac_terms(const DevTables &T, const MacBatch &b, int nterms, int nout, int nq, int first, hipStream_t st,
                   const BasisArg *ba)
{
    if (nterms <= 0 || nterms > HEC_MAC_TERMS || nout <= 0 || nout > HEC_MAC_OUTS) return false;
    if (ba && (!ba->E || ba->nb < 1 || ba->nb > HEC_BASIS_NB || (int)ba->nqp < nq)) return false;
    dim3 g((T.n + EW_THREADS - 1) / EW_THREADS, nq, 1);
    if (ba)
        KLAUNCH("k_mac_terms", (uint64_t)nq * nterms, k_mac_terms_basis, g, dim3(EW_THREADS), 0, st, b, *ba,
                (u32)nterms, (u32)nout, (u32)nq, (u32)first, T);
    else if (nout == 1)
        mac_terms_launch<1>(g, st, b, nterms, nout, nq, first, T);
    else if (nout == 2)
        mac_terms_launch<2>(g, st, b, nterms, nout, nq, first, T);
    else if (nout <= 4)
        mac_terms_launch<4>(g, st, b, nterms, nout, nq, first, T);
    else
        mac_terms_launch<HEC_MAC_OUTS>(g, st, b, nterms, nout, nq, first, T);
    return true;
}

// ModDown tail: out_p[i] = (e_p[i] - y_p[i]) * P^-1 (+ sigma_g(c0)[i] for p = 0)
__global__ void k_moddown_combine(CombineBatch cb, const u64 *c0, u32 nq, u32 nqp, const LevelC *lc,
                                  const u32 *pmap, DevTables T)
{
    const u32 i = blockIdx.y % nq, p = blockIdx.y / nq, r = blockIdx.z;
    const u32 k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= T.n) return;
    const size_t n = T.n;
    const u64 q = T.pc[pmap[i]].q;
    u64 e = cb.e[r][((size_t)p * nqp + i) * n + k];
    u64 y = cb.y[r][((size_t)p * nq + i) * n + k];
    u64 v = shoup_mul(sub_mod(e, y, q), lc->pinv[i], lc->pinv_sh[i], q);
    const u64 *c0r = cb.c0[r] ? cb.c0[r] : c0;
    if (p == 0 && c0r) v = add_mod(v, c0r[(size_t)i * n + auto_src(k, cb.g[r], T.logn)], q);
    if (cb.add[r][p]) v = add_mod(v, cb.add[r][p][(size_t)i * n + k], q);
    cb.out[r][((size_t)p * nq + i) * n + k] = v;
}
void hec_moddown_combine(const DevTables &T, const CombineBatch &cb, int nrot, const u64 *c0, int nq, int nqp,
                         const LevelC *lc, const u32 *pmap, hipStream_t st)
{
    dim3 g((T.n + EW_THREADS - 1) / EW_THREADS, 2 * nq, nrot);
    KLAUNCH("k_moddown_combine", (uint64_t)nrot * 2 * nq, k_moddown_combine, g, dim3(EW_THREADS), 0, st, cb, c0,
            (u32)nq, (u32)nqp, lc, pmap, T);
}

// ---------------------------------------------------------------------------
// rescale
// ---------------------------------------------------------------------------
// tmp[i][t] = (centered last[t]) mod q_i, i < level
__global__ void k_rescale_spread(const u64 *last, u64 *tmp, size_t ls, size_t ts, u32 level, DevTables T)
{
    const u32 i = blockIdx.y, p = blockIdx.z;
    const size_t t = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (t >= T.n) return;
    const u64 ql = T.pc[level].q;
    const PrimeC pc = T.pc[i];
    u64 v = last[p * ls + t];
    u64 r;
    if (v <= (ql - 1) / 2) r = mod64(v, pc);
    else {
        u64 m = mod64(ql - v, pc);
        r = m ? pc.q - m : 0;
    }
    tmp[p * ts + (size_t)i * T.n + t] = r;
}
void hec_rescale_spread(const DevTables &T, const u64 *last_coef, u64 *tmp, size_t last_stride, size_t tmp_stride,
                        int npolys, u32 level, hipStream_t st)
{
    dim3 g((T.n + EW_THREADS - 1) / EW_THREADS, level, npolys);
    hipLaunchKernelGGL(k_rescale_spread, g, dim3(EW_THREADS), 0, st, last_coef, tmp, last_stride, tmp_stride, level, T);
}
__global__ void k_rescale_finish(u64 *out, const u64 *c, const u64 *tmp, size_t so, size_t sc, size_t stt,
                                 const LevelC *lc, DevTables T)
{
    const u32 i = blockIdx.y, p = blockIdx.z;
    const size_t t = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (t >= T.n) return;
    const u64 q = T.pc[i].q;
    const size_t off = (size_t)i * T.n + t;
    out[p * so + off] = shoup_mul(sub_mod(c[p * sc + off], tmp[p * stt + off], q), lc->qlinv[i], lc->qlinv_sh[i], q);
}
void hec_rescale_finish(const DevTables &T, u64 *out, const u64 *c, const u64 *tmp, size_t so, size_t sc,
                        size_t st_, int npolys, u32 level, const LevelC *lc, hipStream_t st)
{
    dim3 g((T.n + EW_THREADS - 1) / EW_THREADS, level, npolys);
    hipLaunchKernelGGL(k_rescale_finish, g, dim3(EW_THREADS), 0, st, out, c, tmp, so, sc, st_, lc, T);
}

// ---------------------------------------------------------------------------
// key assembly and encryption
// ---------------------------------------------------------------------------
__global__ void k_key_finish(u64 *b, u64 *a, const u64 *e, const u64 *sN, const u64 *tgt, const u64 *pm, u32 g,
                             u32 dlo, u32 dhi, const u32 *pmap, DevTables T)
{
    const u32 l = blockIdx.y;
    const u32 k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= T.n) return;
    const u32 pi = pmap[l];
    const PrimeC pc = T.pc[pi];
    const size_t n = T.n, off = (size_t)l * n + k, soff = (size_t)pi * n;
    u64 av = a[off];
    u64 s = sN[soff + k];
    u64 as = mont_mul(av, mont_mul(s, pc.r2, pc.q, pc.qinv_neg), pc.q, pc.qinv_neg);
    u64 v = sub_mod(e[off], as, pc.q);
    if (pm && pi >= dlo && pi < dhi) {
        u64 sg = tgt ? tgt[soff + k] : sN[soff + auto_src(k, g, T.logn)];
        u64 pmm = mont_mul(pm[pi], pc.r2, pc.q, pc.qinv_neg);
        v = add_mod(v, mont_mul(sg, pmm, pc.q, pc.qinv_neg), pc.q);
    }
    b[off] = mont_mul(v, pc.r2, pc.q, pc.qinv_neg);
    a[off] = mont_mul(av, pc.r2, pc.q, pc.qinv_neg);
}
void hec_key_finish(const DevTables &T, u64 *b, u64 *a, const u64 *e, const u64 *sN, const u64 *tgt, const u64 *pm,
                    u32 g, u32 dlo, u32 dhi, int nlimbs, const u32 *pmap, hipStream_t st)
{
    dim3 gr((T.n + EW_THREADS - 1) / EW_THREADS, nlimbs, 1);
    hipLaunchKernelGGL(k_key_finish, gr, dim3(EW_THREADS), 0, st, b, a, e, sN, tgt, pm, g, dlo, dhi, pmap, T);
}

__global__ void k_encrypt_finish(u64 *ct, const u64 *v, const u64 *e0, const u64 *e1, const u64 *m, const u64 *pk,
                                 size_t pks, u32 nq, DevTables T)
{
    const u32 i = blockIdx.y;
    const u32 k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= T.n) return;
    const PrimeC pc = T.pc[i];
    const size_t off = (size_t)i * T.n + k;
    u64 vv = v[off];
    u64 c0 = add_mod(add_mod(mont_mul(vv, pk[off], pc.q, pc.qinv_neg), e0[off], pc.q), m[off], pc.q);
    u64 c1 = add_mod(mont_mul(vv, pk[pks + off], pc.q, pc.qinv_neg), e1[off], pc.q);
    ct[off] = c0;
    ct[(size_t)nq * T.n + off] = c1;
}
void hec_encrypt_finish(const DevTables &T, u64 *ct, const u64 *v, const u64 *e0, const u64 *e1, const u64 *m,
                        const u64 *pk, size_t pk_poly_stride, int nq, hipStream_t st)
{
    dim3 gr((T.n + EW_THREADS - 1) / EW_THREADS, nq, 1);
    hipLaunchKernelGGL(k_encrypt_finish, gr, dim3(EW_THREADS), 0, st, ct, v, e0, e1, m, pk, pk_poly_stride, (u32)nq,
                       T);
}

// ---------------------------------------------------------------------------
// decryption: centered CRT of [nq][n] residues to doubles (Garner mixed radix)
//   v_i = (r_i - sum_{j<i} v_j prod_{k<j} q_k) * (prod_{k<i} q_k)^-1  mod q_i
// value = sum_j v_j prod_{k<j} q_k, centered by comparing the top digit with
// q_top / 2 (for |value| < Q/2 - Q/q_top the test is exact).
// ---------------------------------------------------------------------------
__global__ void k_crt_double(const u64 *res, double *out, u32 nq, const u64 *Mm, const u64 *inv, const u64 *invsh,
                             DevTables T)
{
    const size_t t = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (t >= T.n) return;
    u64 v[HEC_MAX_LIMBS];
    for (u32 i = 0; i < nq; i++) {
        const PrimeC pc = T.pc[i];
        u64 acc = 0;
        for (u32 j = 0; j < i; j++) acc = add_mod(acc, mont_mul(v[j], Mm[i * HEC_MAX_LIMBS + j], pc.q, pc.qinv_neg), pc.q);
        u64 r = res[(size_t)i * T.n + t];
        v[i] = shoup_mul(sub_mod(r, acc, pc.q), inv[i], invsh[i], pc.q);
    }
    const u64 qt = T.pc[nq - 1].q;
    const bool negative = v[nq - 1] >= (qt + 1) / 2;
    double val = 0.0;
    for (int j = (int)nq - 1; j >= 0; j--) {
        u64 q = T.pc[j].q;
        u64 d = negative ? q - 1 - v[j] : v[j];
        val = val * (double)q + (double)d;
    }
    out[t] = negative ? -(val + 1.0) : val;
}
void hec_crt_double(const DevTables &T, const u64 *res, double *out, int nq, const u64 *Mm, const u64 *inv,
                    const u64 *invsh, hipStream_t st)
{
    dim3 g((T.n + EW_THREADS - 1) / EW_THREADS);
    hipLaunchKernelGGL(k_crt_double, g, dim3(EW_THREADS), 0, st, res, out, (u32)nq, Mm, inv, invsh, T);
}

// ---------------------------------------------------------------------------
// products with and sums of constant polynomials (a constant in every slot
// encodes as a constant polynomial, whose evaluations are all equal)
// ---------------------------------------------------------------------------
// op (poly p of out; in read with its own poly stride, so that a ciphertext
// at a higher level can be read as if dropped):
//   SC_MUL  out = in * v_l
//   SC_ADD  out = in + v_l on even polys (c0 of each ciphertext), in on odd ones
//   SC_MAC  out (+)= in * v_l (first: written)
//   SC_DBL_ADD out = 2 in + v_l on even polys, 2 in on odd ones
__global__ void k_scalar(int op, u64 *out, const u64 *in, size_t pso, size_t psi, int first, ScalarArg sa,
                         DevTables T)
{
    const u32 l = blockIdx.y, p = blockIdx.z;
    const size_t t = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (t >= T.n) return;
    const u64 q = T.pc[l].q;
    const size_t lo = (size_t)l * T.n + t;
    const u64 x = in[p * psi + lo];
    u64 *o = out + p * pso + lo;
    switch (op) {
    case SC_MUL: *o = shoup_mul(x, sa.v[l], sa.vsh[l], q); break;
    case SC_ADD: *o = (p & 1) == 0 ? add_mod(x, sa.v[l], q) : x; break;
    case SC_MAC: {
        const u64 y = shoup_mul(x, sa.v[l], sa.vsh[l], q);
        *o = first ? y : add_mod(*o, y, q);
        break;
    }
    case SC_DBL_ADD: {
        const u64 d = add_mod(x, x, q);
        *o = (p & 1) == 0 ? add_mod(d, sa.v[l], q) : d;
        break;
    }
    }
}
void hec_scalar(const DevTables &T, ScalarOp op, u64 *out, const u64 *in, size_t out_poly_stride,
                size_t in_poly_stride, int npolys, int nlimbs, int first, const ScalarArg &sa, hipStream_t st)
{
    if (nlimbs <= 0 || npolys <= 0) return;
    dim3 g((T.n + EW_THREADS - 1) / EW_THREADS, nlimbs, npolys);
    KLAUNCH("k_scalar", (uint64_t)npolys * nlimbs, k_scalar, g, dim3(EW_THREADS), 0, st, (int)op, out, in,
            out_poly_stride, in_poly_stride, first, sa, T);
}

__global__ void __launch_bounds__(EW_THREADS) k_lincomb(u64 *out, size_t pso, LinArg a, u32 nt, DevTables T)
{
    const u32 l = blockIdx.y, p = blockIdx.z;
    const size_t t = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (t >= T.n) return;
    const PrimeC pc = T.pc[l];
    const size_t lo = (size_t)l * T.n + t;
    acc128 acc = {0, 0};
    for (u32 j = 0; j < nt; j++) mac(acc, a.in[j][p * a.ps[j] + lo], a.cm[j][l]);
    out[p * pso + lo] = redc(acc.hi, acc.lo, pc.q, pc.qinv_neg);
}
bool hec_lincomb(const DevTables &T, u64 *out, size_t out_poly_stride, int npolys, int nlimbs, const LinArg &a,
                 int nterms, hipStream_t st)
{
    if (nterms < 1 || nterms > HEC_LIN_TERMS || nlimbs < 1 || nlimbs > HEC_LIN_LIMBS || npolys < 1) return false;
    dim3 g((T.n + EW_THREADS - 1) / EW_THREADS, nlimbs, npolys);
    KLAUNCH("k_lincomb", (uint64_t)npolys * nlimbs, k_lincomb, g, dim3(EW_THREADS), 0, st, out, out_poly_stride, a,
            (u32)nterms, T);
    return true;
}

// ciphertext tensor products in one pass: t_z = [a0 b0][a1 b1][a0 b1 + a1 b0]
// for pair z = blockIdx.z (all plain evaluation form; b taken into Montgomery
// form in registers)
__global__ void __launch_bounds__(EW_THREADS) k_tensor(u64 *t, const u64 *a, const u64 *b, size_t P, DevTables T)
{
    const u32 l = blockIdx.y, z = blockIdx.z;
    const size_t k = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= T.n) return;
    const PrimeC pc = T.pc[l];
    const size_t off = (size_t)l * T.n + k;
    a += 2 * z * P;
    b += 2 * z * P;
    t += 3 * z * P;
    const u64 a0 = a[off], a1 = a[P + off];
    const u64 b0 = mont_mul(b[off], pc.r2, pc.q, pc.qinv_neg), b1 = mont_mul(b[P + off], pc.r2, pc.q, pc.qinv_neg);
    t[off] = mont_mul(a0, b0, pc.q, pc.qinv_neg);
    t[P + off] = mont_mul(a1, b1, pc.q, pc.qinv_neg);
    t[2 * P + off] = add_mod(mont_mul(a0, b1, pc.q, pc.qinv_neg), mont_mul(a1, b0, pc.q, pc.qinv_neg), pc.q);
}
__global__ void __launch_bounds__(EW_THREADS) k_tensor_items(u64 *t, TensorItems it, u32 per, size_t P, DevTables T)
{
    const u32 l = blockIdx.y, z = blockIdx.z;
    const size_t k = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= T.n) return;
    const PrimeC pc = T.pc[l];
    const size_t off = (size_t)l * T.n + k;
    const u64 *a = it.a[z / per] + 2 * (z % per) * P, *b = it.b[z / per] + 2 * (z % per) * P;
    t += 3 * z * P;
    const u64 a0 = a[off], a1 = a[P + off];
    const u64 b0 = mont_mul(b[off], pc.r2, pc.q, pc.qinv_neg), b1 = mont_mul(b[P + off], pc.r2, pc.q, pc.qinv_neg);
    t[off] = mont_mul(a0, b0, pc.q, pc.qinv_neg);
    t[P + off] = mont_mul(a1, b1, pc.q, pc.qinv_neg);
    t[2 * P + off] = add_mod(mont_mul(a0, b1, pc.q, pc.qinv_neg), mont_mul(a1, b0, pc.q, pc.qinv_neg), pc.q);
}
bool hec_tensor_items(const DevTables &T, u64 *t, const TensorItems &it, int nitems, int per, int nq, hipStream_t st)
{
    if (nitems < 1 || nitems > HEC_TENSOR_ITEMS || per < 1 || nq < 1) return false;
    dim3 g((T.n + EW_THREADS - 1) / EW_THREADS, nq, nitems * per);
    KLAUNCH("k_tensor", (uint64_t)nq * nitems * per, k_tensor_items, g, dim3(EW_THREADS), 0, st, t, it, (u32)per,
            (size_t)nq * T.n, T);
    return true;
}
void hec_tensor(const DevTables &T, u64 *t, const u64 *a, const u64 *b, int nq, int cnt, hipStream_t st)
{
    if (cnt <= 0) return;
    dim3 g((T.n + EW_THREADS - 1) / EW_THREADS, nq, cnt);
    KLAUNCH("k_tensor", (uint64_t)nq * cnt, k_tensor, g, dim3(EW_THREADS), 0, st, t, a, b, (size_t)nq * T.n, T);
}

// Bandwidth probe: `nr` streams of `words` u64 read and `nw` written, one word
// of each per lane, non-temporal, plain grid order -- the access mix of a
// streaming kernel without its arithmetic (every output word depends on every
// word read, so no load is dropped).
__global__ void __launch_bounds__(EW_THREADS) k_probe_stream(const u64 *in, u64 *out, size_t words, u32 nr, u32 nw)
{
    const size_t k = (size_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= words) return;
    u64 v[HEC_PROBE_MAX_READ];
#pragma unroll
    for (u32 r = 0; r < HEC_PROBE_MAX_READ; r++)
        if (r < nr) v[r] = __builtin_nontemporal_load(in + (size_t)r * words + k);
    u64 x = 0;
#pragma unroll
    for (u32 r = 0; r < HEC_PROBE_MAX_READ; r++)
        if (r < nr) x += v[r];
    for (u32 w = 0; w < nw; w++) __builtin_nontemporal_store(x + w, out + (size_t)w * words + k);
}
void hec_probe_stream(const u64 *in, u64 *out, size_t words, int nr, int nw, hipStream_t st)
{
    dim3 g((u32)((words + EW_THREADS - 1) / EW_THREADS));
    hipLaunchKernelGGL(k_probe_stream, g, dim3(EW_THREADS), 0, st, in, out, words, (u32)nr, (u32)nw);
}
