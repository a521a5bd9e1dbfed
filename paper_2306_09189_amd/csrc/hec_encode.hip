// hec_encode.hip -- CKKS encoding and decoding on the GPU (canonical embedding
// of the real slots, Background: CKKS encoding).
//
// Encoding of slot values z_j (j < N = n/2) into integer coefficients:
//   m_t = round( (scale / n) * Re( sum_k v_k exp(-2 pi i k t / n) exp(-i pi t / n) ) )
// where v holds z_j at the positions of the roots zeta^(5^j) and zeta^(-5^j)
// (k = (5^j mod 2n - 1)/2 and n - 1 - k).  The transform runs in double-double
// arithmetic (about 106 bits) as an in-place radix-2 decimation-in-time FFT,
// so the integer rounding decides on a value within ~2^-100 relative of the
// exact one.  Decoding is the conjugate transform in plain double precision.
//
// Double-double arithmetic relies on exactly rounded IEEE operations in a
// fixed order: contraction into FMA is disabled for this file, and the one
// FMA that is wanted (the error term of a product) is written explicitly.
#include "hec_common.h"

#pragma clang fp contract(off)

#define DEV __device__ __forceinline__
#define ENC_THREADS 256
#define ENC_LDS_LOG 11  // 2^11 points of 32 bytes (64 KiB) per block for the first stages

namespace {
struct dd {
    double h, l;
};
DEV dd two_sum(double a, double b)
{
    double s = a + b, bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
DEV dd quick(double a, double b)
{
    double s = a + b;
    return {s, b - (s - a)};
}
DEV dd two_prod(double a, double b)
{
    double p = a * b;
    return {p, fma(a, b, -p)};
}
DEV dd add(dd x, dd y)
{
    dd s = two_sum(x.h, y.h), t = two_sum(x.l, y.l);
    s.l += t.h;
    s = quick(s.h, s.l);
    s.l += t.l;
    return quick(s.h, s.l);
}
DEV dd neg(dd x) { return {-x.h, -x.l}; }
DEV dd sub(dd x, dd y) { return add(x, neg(y)); }
DEV dd mul(dd x, dd y)
{
    dd p = two_prod(x.h, y.h);
    p.l += x.h * y.l + x.l * y.h;
    return quick(p.h, p.l);
}
DEV dd mul_d(dd x, double d)
{
    dd p = two_prod(x.h, d);
    p.l += x.l * d;
    return quick(p.h, p.l);
}
// complex double-double value of one FFT point
struct cdd {
    dd re, im;
};
DEV cdd ld_c(const double4 *p)
{
    double4 v = *p;
    return {{v.x, v.y}, {v.z, v.w}};
}
DEV void st_c(double4 *p, cdd c) { *p = make_double4(c.re.h, c.re.l, c.im.h, c.im.l); }
DEV u32 brev_n(u32 x, u32 logn) { return __brev(x) >> (32 - logn); }

// butterfly of the decimation-in-time stage with half-length h: twiddle
// exp(-2 pi i j / (2h)) = cos - i sin of angle index e = j * (n / h) in units of pi / n
DEV void bfly(cdd &a, cdd &b, const double4 *tw, u32 j, u32 e)
{
    cdd v = b;
    if (j) {
        double4 w = tw[e];
        dd wr = {w.x, w.y}, wi = {-w.z, -w.w};
        v.re = sub(mul(b.re, wr), mul(b.im, wi));
        v.im = add(mul(b.re, wi), mul(b.im, wr));
    }
    cdd x = a;
    a.re = add(x.re, v.re);
    a.im = add(x.im, v.im);
    b.re = sub(x.re, v.re);
    b.im = sub(x.im, v.im);
}

// round half away from zero of a double-double; *bad set when |x| >= 2^62
DEV int64_t round_away(dd x, int *bad)
{
    if (!(fabs(x.h) < 4611686018427387904.0)) {
        *bad = 1;
        return 0;
    }
    double f = floor(x.h);
    double frac = (x.h - f) + x.l;
    int64_t base = (int64_t)f;
    while (frac >= 1.0) {
        frac -= 1.0;
        base += 1;
    }
    while (frac < 0.0) {
        frac += 1.0;
        base -= 1;
    }
    if (frac > 0.5) return base + 1;
    if (frac < 0.5) return base;
    return base >= 0 ? base + 1 : base;
}
}  // namespace

// v in bit-reversed order: point brv(k) <- z_j for k = root(j) and n-1-root(j); imaginary parts 0.
// Grid (N / ENC_THREADS, count); block (0, 0) also clears the overflow flag.
__global__ void __launch_bounds__(ENC_THREADS) k_enc_scatter(const double *z, size_t zstride, u32 nz,
                                                             const u32 *root, double4 *buf, u32 logn, int *flag)
{
    const u32 N = 1u << (logn - 1), j = blockIdx.x * ENC_THREADS + threadIdx.x;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *flag = 0;
    if (j >= N) return;
    const double v = j < nz ? z[blockIdx.y * zstride + j] : 0.0;
    double4 *b = buf + ((size_t)blockIdx.y << logn);
    const u32 k = root[j];
    b[brev_n(k, logn)] = make_double4(v, 0.0, 0.0, 0.0);
    b[brev_n((1u << logn) - 1 - k, logn)] = make_double4(v, 0.0, 0.0, 0.0);
}

// stages h = 1 .. 2^(c-1) inside contiguous chunks of 2^c points, in LDS
__global__ void __launch_bounds__(ENC_THREADS) k_enc_stages_lds(double4 *buf, const double4 *tw, u32 logn, u32 c)
{
    __shared__ double4 s[1u << ENC_LDS_LOG];
    const u32 C = 1u << c;
    double4 *b = buf + ((size_t)blockIdx.y << logn) + (size_t)blockIdx.x * C;
    for (u32 e = threadIdx.x; e < C; e += ENC_THREADS) s[e] = b[e];
    __syncthreads();
    for (u32 lh = 0; lh < c; lh++) {
        const u32 h = 1u << lh;
        for (u32 t = threadIdx.x; t < C / 2; t += ENC_THREADS) {
            const u32 j = t & (h - 1), i = (t >> lh) << (lh + 1);
            cdd a = ld_c(&s[i + j]), bb = ld_c(&s[i + j + h]);
            bfly(a, bb, tw, j, j << (logn - lh));
            st_c(&s[i + j], a);
            st_c(&s[i + j + h], bb);
        }
        __syncthreads();
    }
    for (u32 e = threadIdx.x; e < C; e += ENC_THREADS) b[e] = s[e];
}

// one stage with half-length h = 2^lh over the whole transform
__global__ void __launch_bounds__(ENC_THREADS) k_enc_stage(double4 *buf, const double4 *tw, u32 logn, u32 lh)
{
    const u32 t = blockIdx.x * ENC_THREADS + threadIdx.x;
    if (t >= (1u << (logn - 1))) return;
    const u32 h = 1u << lh, j = t & (h - 1), i = (t >> lh) << (lh + 1);
    double4 *b = buf + ((size_t)blockIdx.y << logn);
    cdd a = ld_c(&b[i + j]), bb = ld_c(&b[i + j + h]);
    bfly(a, bb, tw, j, j << (logn - lh));
    st_c(&b[i + j], a);
    st_c(&b[i + j + h], bb);
}

// m_t = round((scale / n) * (re_t cos(pi t / n) + im_t sin(pi t / n)))
__global__ void __launch_bounds__(ENC_THREADS) k_enc_finish(const double4 *buf, const double4 *tw, double sc,
                                                            int64_t *m, u32 logn, int *flag)
{
    const u32 t = blockIdx.x * ENC_THREADS + threadIdx.x;
    if (t >= (1u << logn)) return;
    const size_t off = ((size_t)blockIdx.y << logn) + t;
    const cdd x = ld_c(&buf[off]);
    const double4 w = tw[t];
    const dd v = add(mul(x.re, dd{w.x, w.y}), mul(x.im, dd{w.z, w.w}));
    int bad = 0;
    m[off] = round_away(mul_d(v, sc), &bad);
    if (bad) atomicOr(flag, 1);
}

void hec_encode(const double *z, size_t zstride, u32 nz, u32 count, double scale, const u32 *root,
                const double4 *tw, double4 *work, int64_t *m, int *flag, u32 logn, hipStream_t st)
{
    const u32 n = 1u << logn, N = n / 2;
    hipLaunchKernelGGL(k_enc_scatter, dim3((N + ENC_THREADS - 1) / ENC_THREADS, count), dim3(ENC_THREADS), 0, st,
                       z, zstride, nz, root, work, logn, flag);
    const u32 c = logn < ENC_LDS_LOG ? logn : ENC_LDS_LOG;
    hipLaunchKernelGGL(k_enc_stages_lds, dim3(n >> c, count), dim3(ENC_THREADS), 0, st, work, tw, logn, c);
    for (u32 lh = c; lh < logn; lh++)
        hipLaunchKernelGGL(k_enc_stage, dim3((N + ENC_THREADS - 1) / ENC_THREADS, count), dim3(ENC_THREADS), 0, st,
                           work, tw, logn, lh);
    hipLaunchKernelGGL(k_enc_finish, dim3((n + ENC_THREADS - 1) / ENC_THREADS, count), dim3(ENC_THREADS), 0, st,
                       work, tw, scale / (double)n, m, logn, flag);
}

// ---------------------------------------------------------------------------
// decoding: z_j = (1/scale) Re( sum_t m_t exp(i pi t / n) exp(2 pi i t k_j / n) ) at k_j = root(j)
// (double precision; the result is compared within a tolerance, never rounded to an integer)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(ENC_THREADS) k_dec_scatter(const double *m, const double4 *tw, double2 *a,
                                                             u32 logn)
{
    const u32 t = blockIdx.x * ENC_THREADS + threadIdx.x;
    if (t >= (1u << logn)) return;
    const double4 w = tw[t];
    a[brev_n(t, logn)] = make_double2(m[t] * w.x, m[t] * w.z);
}

// stages in LDS for contiguous chunks of 2^c points (inverse direction: twiddle exp(+2 pi i j / (2h)))
__global__ void __launch_bounds__(ENC_THREADS) k_dec_stages_lds(double2 *a, const double4 *tw, u32 logn, u32 c)
{
    __shared__ double2 s[1u << (ENC_LDS_LOG + 1)];
    const u32 C = 1u << c;
    double2 *b = a + (size_t)blockIdx.x * C;
    for (u32 e = threadIdx.x; e < C; e += ENC_THREADS) s[e] = b[e];
    __syncthreads();
    for (u32 lh = 0; lh < c; lh++) {
        const u32 h = 1u << lh;
        for (u32 t = threadIdx.x; t < C / 2; t += ENC_THREADS) {
            const u32 j = t & (h - 1), i = (t >> lh) << (lh + 1);
            const double4 w = tw[j << (logn - lh)];
            const double2 u = s[i + j], x = s[i + j + h];
            const double2 v = make_double2(x.x * w.x - x.y * w.z, x.x * w.z + x.y * w.x);
            s[i + j] = make_double2(u.x + v.x, u.y + v.y);
            s[i + j + h] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
    for (u32 e = threadIdx.x; e < C; e += ENC_THREADS) b[e] = s[e];
}

__global__ void __launch_bounds__(ENC_THREADS) k_dec_stage(double2 *a, const double4 *tw, u32 logn, u32 lh)
{
    const u32 t = blockIdx.x * ENC_THREADS + threadIdx.x;
    if (t >= (1u << (logn - 1))) return;
    const u32 h = 1u << lh, j = t & (h - 1), i = (t >> lh) << (lh + 1);
    const double4 w = tw[j << (logn - lh)];
    const double2 u = a[i + j], x = a[i + j + h];
    const double2 v = make_double2(x.x * w.x - x.y * w.z, x.x * w.z + x.y * w.x);
    a[i + j] = make_double2(u.x + v.x, u.y + v.y);
    a[i + j + h] = make_double2(u.x - v.x, u.y - v.y);
}

__global__ void __launch_bounds__(ENC_THREADS) k_dec_gather(const double2 *a, const u32 *root, double scale,
                                                            double *z, u32 nz)
{
    const u32 j = blockIdx.x * ENC_THREADS + threadIdx.x;
    if (j >= nz) return;
    z[j] = a[root[j]].x / scale;
}

void hec_decode(const double *m, double scale, const u32 *root, const double4 *tw, double2 *work, double *z,
                u32 nz, u32 logn, hipStream_t st)
{
    const u32 n = 1u << logn, N = n / 2;
    hipLaunchKernelGGL(k_dec_scatter, dim3((n + ENC_THREADS - 1) / ENC_THREADS), dim3(ENC_THREADS), 0, st, m, tw,
                       work, logn);
    const u32 c = logn < ENC_LDS_LOG + 1 ? logn : ENC_LDS_LOG + 1;
    hipLaunchKernelGGL(k_dec_stages_lds, dim3(n >> c), dim3(ENC_THREADS), 0, st, work, tw, logn, c);
    for (u32 lh = c; lh < logn; lh++)
        hipLaunchKernelGGL(k_dec_stage, dim3((N + ENC_THREADS - 1) / ENC_THREADS), dim3(ENC_THREADS), 0, st, work,
                           tw, logn, lh);
    if (nz)
        hipLaunchKernelGGL(k_dec_gather, dim3((nz + ENC_THREADS - 1) / ENC_THREADS), dim3(ENC_THREADS), 0, st, work,
                           root, scale, z, nz);
}
