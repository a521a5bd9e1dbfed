/*
 * ckks_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, CPU reference of the RNS-CKKS arithmetic that the homomorphic
 * convolution and average pooling of "High-Resolution Convolutional Neural
 * Networks on Homomorphically Encrypted Data via Sharding Ciphertexts"
 * (Maloney et al., arXiv 2306.09189) are built on.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library; the
 * product path never does.  It shares no code, header or table with the GPU
 * library.
 *
 * The paper (Background, "Homomorphic encryption") fixes the ring
 * Z_Q[x]/(x^n + 1) with n = 2N and N real slots, levels consumed by
 * multiplication, and cyclic slot rotations; it uses RNS-CKKS through a
 * library and does not spell out the scheme.  The scheme steps below are the
 * standard RNS-CKKS ones (encoding by the canonical embedding, public-key
 * encryption, hybrid key switching with fast base conversion, rescale), each
 * written out in the plainest form:
 *   - every modular product is (unsigned __int128)a*b % q; no Barrett, no
 *     Shoup, no Montgomery;
 *   - polynomials live in coefficient form; a product of two polynomials goes
 *     through a textbook negacyclic NTT that the tests pin to the schoolbook
 *     product;
 *   - the encoder works in IEEE binary128 (__float128).
 * Parity is pinned by the tests under tests/ (schoolbook products, big-integer
 * CRT, RFC 8439 ChaCha20 vectors, slot-rotation invariants).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <quadmath.h>

typedef unsigned __int128 u128;
typedef __float128 f128;

#define ORC_MAXP 96

/* Parameters of one RNS-CKKS instance.
 * mod[0..L]       : ciphertext primes q_0..q_L
 * mod[L+1..L+k]   : special primes p_0..p_{k-1} of the key-switching modulus P
 * Digits of the hybrid key switch are consecutive runs of alpha primes of
 * q_0..q_L; dnum = ceil((L+1)/alpha). */
typedef struct {
    uint32_t logn, n;
    uint32_t L, k, dnum, alpha;
    uint64_t mod[ORC_MAXP];
    uint64_t psi[ORC_MAXP]; /* a primitive 2n-th root of unity mod each prime */
} orc_params;

/* ------------------------------------------------------------------ */
/* modular arithmetic                                                  */
/* ------------------------------------------------------------------ */

uint64_t orc_mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + b) % q); }
static uint64_t submod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + q - b) % q); }

uint64_t orc_powmod(uint64_t a, uint64_t e, uint64_t q)
{
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = orc_mulmod(r, a, q);
        a = orc_mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}

/* inverse modulo a prime, by Fermat's little theorem */
uint64_t orc_invmod(uint64_t a, uint64_t q) { return orc_powmod(a, q - 2, q); }

/* Deterministic Miller-Rabin: the first twelve primes as bases decide every
 * 64-bit integer. */
int orc_is_prime(uint64_t m)
{
    static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (m < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (m == bases[i]) return 1;
        if (m % bases[i] == 0) return 0;
    }
    uint64_t d = m - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        uint64_t x = orc_powmod(bases[i], d, m);
        if (x == 1 || x == m - 1) continue;
        int composite = 1;
        for (int r = 1; r < s; r++) {
            x = orc_mulmod(x, x, m);
            if (x == m - 1) { composite = 0; break; }
        }
        if (composite) return 0;
    }
    return 1;
}

/* The prime chain: for a requested bit size b, candidates 2^b - j*2n + 1 for
 * j = 1, 2, ... (so every candidate is below 2^b and is 1 mod 2n, which an
 * n-point negacyclic NTT needs); the first prime not already taken is used. */
uint64_t orc_find_prime(uint32_t bits, uint32_t n, const uint64_t *taken, uint32_t ntaken)
{
    uint64_t step = 2ull * n;
    for (uint64_t j = 1;; j++) {
        uint64_t c = (1ull << bits) - j * step + 1;
        if (c < (1ull << (bits - 1))) return 0;
        if (!orc_is_prime(c)) continue;
        int used = 0;
        for (uint32_t t = 0; t < ntaken; t++)
            if (taken[t] == c) used = 1;
        if (!used) return c;
    }
}

/* psi = x^((q-1)/2n) for the smallest x >= 2 for which that power has
 * psi^n = -1, i.e. order exactly 2n. */
uint64_t orc_find_psi(uint64_t q, uint32_t n)
{
    for (uint64_t x = 2;; x++) {
        uint64_t g = orc_powmod(x, (q - 1) / (2ull * n), q);
        if (orc_powmod(g, n, q) == q - 1) return g;
    }
}

int orc_params_init(orc_params *p, uint32_t logn, uint32_t nq, const uint32_t *qbits, uint32_t k,
                    const uint32_t *pbits, uint32_t dnum)
{
    if (logn < 2 || logn > 17 || nq < 1 || nq + k > ORC_MAXP || dnum < 1 || dnum > nq) return -1;
    memset(p, 0, sizeof(*p));
    p->logn = logn;
    p->n = 1u << logn;
    p->L = nq - 1;
    p->k = k;
    p->alpha = (nq + dnum - 1) / dnum;
    p->dnum = (nq + p->alpha - 1) / p->alpha;
    uint32_t cnt = 0;
    for (uint32_t i = 0; i < nq + k; i++) {
        uint32_t b = i < nq ? qbits[i] : pbits[i - nq];
        if (b < 20 || b > 61) return -2;
        uint64_t q = orc_find_prime(b, p->n, p->mod, cnt);
        if (!q) return -3;
        p->mod[cnt] = q;
        p->psi[cnt] = orc_find_psi(q, p->n);
        cnt++;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* negacyclic NTT: a_hat[k] = a(psi^(2k+1)) = sum_t a[t] psi^((2k+1)t)  */
/* ------------------------------------------------------------------ */

static void bitrev_permute(uint64_t *a, uint32_t n)
{
    for (uint32_t i = 1, j = 0; i < n; i++) {
        uint32_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { uint64_t t = a[i]; a[i] = a[j]; a[j] = t; }
    }
}

/* in-place cyclic DFT of length n with root w (radix-2, decimation in time) */
static void cyclic_dft(uint64_t *a, uint32_t n, uint64_t q, uint64_t w)
{
    bitrev_permute(a, n);
    for (uint32_t len = 2; len <= n; len <<= 1) {
        uint64_t wl = orc_powmod(w, n / len, q);
        for (uint32_t i = 0; i < n; i += len) {
            uint64_t x = 1;
            for (uint32_t j = 0; j < len / 2; j++) {
                uint64_t u = a[i + j], v = orc_mulmod(a[i + j + len / 2], x, q);
                a[i + j] = addmod(u, v, q);
                a[i + j + len / 2] = submod(u, v, q);
                x = orc_mulmod(x, wl, q);
            }
        }
    }
}

/* forward: twist by psi^t, then the cyclic DFT with omega = psi^2 */
void orc_ntt(uint64_t *a, uint32_t n, uint64_t q, uint64_t psi)
{
    uint64_t x = 1;
    for (uint32_t t = 0; t < n; t++) { a[t] = orc_mulmod(a[t], x, q); x = orc_mulmod(x, psi, q); }
    cyclic_dft(a, n, q, orc_mulmod(psi, psi, q));
}

/* inverse: cyclic DFT with omega^-1, divide by n, untwist by psi^-t */
void orc_intt(uint64_t *a, uint32_t n, uint64_t q, uint64_t psi)
{
    uint64_t ipsi = orc_invmod(psi, q);
    cyclic_dft(a, n, q, orc_mulmod(ipsi, ipsi, q));
    uint64_t ninv = orc_invmod(n % q, q), x = ninv;
    for (uint32_t t = 0; t < n; t++) { a[t] = orc_mulmod(a[t], x, q); x = orc_mulmod(x, ipsi, q); }
}

/* out = a * b in Z_q[x]/(x^n + 1) */
void orc_polymul(const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t n, uint64_t q, uint64_t psi)
{
    uint64_t *ta = malloc(sizeof(uint64_t) * n), *tb = malloc(sizeof(uint64_t) * n);
    memcpy(ta, a, sizeof(uint64_t) * n);
    memcpy(tb, b, sizeof(uint64_t) * n);
    orc_ntt(ta, n, q, psi);
    orc_ntt(tb, n, q, psi);
    for (uint32_t i = 0; i < n; i++) ta[i] = orc_mulmod(ta[i], tb[i], q);
    orc_intt(ta, n, q, psi);
    memcpy(out, ta, sizeof(uint64_t) * n);
    free(ta);
    free(tb);
}

/* ------------------------------------------------------------------ */
/* ChaCha20 (RFC 8439) keystream and the samplers built on it          */
/* ------------------------------------------------------------------ */

static uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

#define QR(a, b, c, d)                                                                                             \
    do {                                                                                                           \
        a += b; d ^= a; d = rotl32(d, 16);                                                                         \
        c += d; b ^= c; b = rotl32(b, 12);                                                                         \
        a += b; d ^= a; d = rotl32(d, 8);                                                                          \
        c += d; b ^= c; b = rotl32(b, 7);                                                                          \
    } while (0)

/* RFC 8439 section 2.3: the ChaCha20 block function */
void orc_chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3], uint32_t out[16])
{
    uint32_t s[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u,
                      key[0], key[1], key[2], key[3], key[4], key[5], key[6], key[7],
                      counter, nonce[0], nonce[1], nonce[2]};
    uint32_t x[16];
    memcpy(x, s, sizeof(x));
    for (int i = 0; i < 10; i++) {
        QR(x[0], x[4], x[8], x[12]);
        QR(x[1], x[5], x[9], x[13]);
        QR(x[2], x[6], x[10], x[14]);
        QR(x[3], x[7], x[11], x[15]);
        QR(x[0], x[5], x[10], x[15]);
        QR(x[1], x[6], x[11], x[12]);
        QR(x[2], x[7], x[8], x[13]);
        QR(x[3], x[4], x[9], x[14]);
    }
    for (int i = 0; i < 16; i++) out[i] = x[i] + s[i];
}

/* The randomness convention: a stream is named by (seed, purpose, index).
 * ChaCha20 key = the 64-bit seed little-endian followed by 24 zero bytes;
 * nonce = purpose (u32) then index (u64), little-endian; the block counter
 * starts at 0.  Word w of the stream is the little-endian u64 at byte 8w of
 * the keystream (block w/8, 32-bit words 2(w%8) and 2(w%8)+1). */
void orc_stream_u64(uint64_t seed, uint32_t purpose, uint64_t index, uint64_t first, uint64_t count, uint64_t *out)
{
    uint32_t key[8] = {(uint32_t)seed, (uint32_t)(seed >> 32), 0, 0, 0, 0, 0, 0};
    uint32_t nonce[3] = {purpose, (uint32_t)index, (uint32_t)(index >> 32)};
    uint32_t blk[16];
    uint64_t cur = UINT64_MAX;
    for (uint64_t i = 0; i < count; i++) {
        uint64_t w = first + i;
        if (w / 8 != cur) {
            cur = w / 8;
            orc_chacha20_block(key, (uint32_t)cur, nonce, blk);
        }
        uint32_t lo = blk[2 * (w % 8)], hi = blk[2 * (w % 8) + 1];
        out[i] = (uint64_t)lo | ((uint64_t)hi << 32);
    }
}

/* Uniform residues: coefficient c of the stream (c = limb*n + t) takes words
 * 2c and 2c+1 as a 128-bit integer hi:lo and reduces it mod q.  Fixed-length
 * draws keep the word position of every coefficient fixed. */
void orc_sample_uniform(const orc_params *p, uint64_t seed, uint32_t purpose, uint64_t index,
                        const uint32_t *pidx, uint32_t nl, uint64_t *out)
{
    uint32_t n = p->n;
#pragma omp parallel for
    for (uint32_t l = 0; l < nl; l++) {
        uint64_t *w = malloc(sizeof(uint64_t) * 2 * n);
        orc_stream_u64(seed, purpose, index, 2ull * l * n, 2ull * n, w);
        uint64_t q = p->mod[pidx[l]];
        for (uint32_t t = 0; t < n; t++) {
            u128 v = ((u128)w[2 * t] << 64) | w[2 * t + 1];
            out[(size_t)l * n + t] = (uint64_t)(v % q);
        }
        free(w);
    }
}

/* Ternary: word t gives (w mod 3) - 1. */
void orc_sample_ternary(uint64_t seed, uint32_t purpose, uint64_t index, uint32_t n, int64_t *out)
{
    uint64_t *w = malloc(sizeof(uint64_t) * n);
    orc_stream_u64(seed, purpose, index, 0, n, w);
    for (uint32_t t = 0; t < n; t++) out[t] = (int64_t)(w[t] % 3) - 1;
    free(w);
}

/* Discrete Gaussian, sigma = 3.2, support |x| <= 19 (about 6 sigma), by
 * cumulative-table inversion.  Word t: bit 0 is the sign, the upper 63 bits
 * v select the magnitude k = min{k : v < T[k]} with
 * T[k] = floor(2^63 * sum_{i<=k} w_i / sum_i w_i), w_0 = 1,
 * w_i = 2 exp(-i^2 / (2 sigma^2)) (both signs of i).  The table is built here
 * in binary128. */
#define ORC_GAUSS_K 19
void orc_gauss_table(double sigma, uint64_t *T)
{
    f128 w[ORC_GAUSS_K + 1], tot = 0;
    for (int i = 0; i <= ORC_GAUSS_K; i++) {
        w[i] = (i == 0 ? 1 : 2) * expq(-(f128)(i * i) / (2 * (f128)sigma * (f128)sigma));
        tot += w[i];
    }
    f128 acc = 0;
    for (int i = 0; i < ORC_GAUSS_K; i++) {
        acc += w[i];
        T[i] = (uint64_t)floorq(acc / tot * 9223372036854775808.0Q);
    }
}

void orc_sample_gauss(uint64_t seed, uint32_t purpose, uint64_t index, uint32_t n, double sigma, int64_t *out)
{
    uint64_t T[ORC_GAUSS_K];
    orc_gauss_table(sigma, T);
    uint64_t *w = malloc(sizeof(uint64_t) * n);
    orc_stream_u64(seed, purpose, index, 0, n, w);
    for (uint32_t t = 0; t < n; t++) {
        uint64_t v = w[t] >> 1;
        int64_t mag = ORC_GAUSS_K;
        for (int i = 0; i < ORC_GAUSS_K; i++)
            if (v < T[i]) { mag = i; break; }
        out[t] = (w[t] & 1) ? -mag : mag;
    }
    free(w);
}

/* ------------------------------------------------------------------ */
/* encoding: canonical embedding restricted to real slots              */
/* ------------------------------------------------------------------ */

/* Slot j of a plaintext m(x) is m(zeta^(5^j mod 2n)) with zeta = exp(i pi/n),
 * j < N = n/2; the conjugate roots zeta^(-5^j) hold the same real value.  The
 * encoding of real z at scale s is therefore
 *   m_t = round(s * (2/n) * sum_j z_j cos(pi * (5^j t mod 2n) / n)),
 * rounded half away from zero.  Decoding is z_j = (1/s) sum_t m_t
 * cos(pi (5^j t mod 2n) / n).  Both are computed in binary128. */

static int64_t round_half_away(f128 x, int *overflow)
{
    f128 r = x < 0 ? -floorq(-x + 0.5Q) : floorq(x + 0.5Q);
    if (fabsq(r) > 4611686018427387904.0Q) { *overflow = 1; return 0; }
    return (int64_t)r;
}

/* the plain definition, O(n*N): used to pin the FFT form on small rings */
int orc_encode_direct(uint32_t n, const double *z, uint32_t nz, double scale, int64_t *m)
{
    uint32_t N = n / 2, twon = 2 * n;
    f128 *c = malloc(sizeof(f128) * twon);
    for (uint32_t e = 0; e < twon; e++) c[e] = cosq(M_PIq * (f128)e / (f128)n);
    uint64_t *five = malloc(sizeof(uint64_t) * N);
    uint64_t f = 1;
    for (uint32_t j = 0; j < N; j++) { five[j] = f; f = f * 5 % twon; }
    int overflow = 0;
    for (uint32_t t = 0; t < n; t++) {
        f128 acc = 0;
        for (uint32_t j = 0; j < nz && j < N; j++) acc += (f128)z[j] * c[(five[j] * t) % twon];
        m[t] = round_half_away((f128)scale * 2 * acc / (f128)n, &overflow);
    }
    free(c);
    free(five);
    return overflow ? -1 : 0;
}

/* cos/sin(2 pi k / n) for k < n and cos/sin(pi t / n) for t < n, cached for
 * the last ring size used (the tables are pure functions of n) */
static uint32_t roots_n;
static f128 *roots_c, *roots_s, *half_c, *half_s;
static void unit_roots(uint32_t n, const f128 **c, const f128 **s)
{
    if (roots_n != n) {
        free(roots_c); free(roots_s); free(half_c); free(half_s);
        roots_c = malloc(sizeof(f128) * n); roots_s = malloc(sizeof(f128) * n);
        half_c = malloc(sizeof(f128) * n); half_s = malloc(sizeof(f128) * n);
        for (uint32_t k = 0; k < n; k++) {
            roots_c[k] = cosq(2 * M_PIq * (f128)k / (f128)n);
            roots_s[k] = sinq(2 * M_PIq * (f128)k / (f128)n);
            half_c[k] = cosq(M_PIq * (f128)k / (f128)n);
            half_s[k] = sinq(M_PIq * (f128)k / (f128)n);
        }
        roots_n = n;
    }
    *c = roots_c;
    *s = roots_s;
}

/* radix-2 complex DFT in binary128: X[k] = sum_t x[t] exp(sign * 2 pi i k t / n) */
static void qdft(f128 *re, f128 *im, uint32_t n, int sign)
{
    for (uint32_t i = 1, j = 0; i < n; i++) {
        uint32_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            f128 t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
    const f128 *cr, *ci0;
    unit_roots(n, &cr, &ci0);
    for (uint32_t len = 2; len <= n; len <<= 1) {
        uint32_t stride = n / len;
        for (uint32_t i = 0; i < n; i += len)
            for (uint32_t j = 0; j < len / 2; j++) {
                f128 wr = cr[j * stride], wi = sign * ci0[j * stride];
                uint32_t a = i + j, b = i + j + len / 2;
                f128 vr = re[b] * wr - im[b] * wi, vi = re[b] * wi + im[b] * wr;
                re[b] = re[a] - vr; im[b] = im[a] - vi;
                re[a] += vr; im[a] += vi;
            }
    }
}

/* The same encoding through a length-n DFT over the odd powers of zeta:
 * with v[k] the value at zeta^(2k+1), m_t = (s/n) Re(zeta^-t sum_k v[k] omega^-kt),
 * omega = zeta^2. */
int orc_encode(uint32_t n, const double *z, uint32_t nz, double scale, int64_t *m)
{
    uint32_t N = n / 2, twon = 2 * n;
    f128 *re = calloc(n, sizeof(f128)), *im = calloc(n, sizeof(f128));
    uint64_t f = 1;
    for (uint32_t j = 0; j < N; j++) {
        f128 v = j < nz ? (f128)z[j] : 0;
        re[(f - 1) / 2] = v;            /* root zeta^(5^j)  */
        re[(twon - f - 1) / 2] = v;     /* root zeta^(-5^j) */
        f = f * 5 % twon;
    }
    qdft(re, im, n, -1);
    int overflow = 0;
    for (uint32_t t = 0; t < n; t++) {
        /* Re((re + i im) * exp(-i pi t / n)) */
        f128 val = re[t] * half_c[t] + im[t] * half_s[t];
        m[t] = round_half_away((f128)scale * val / (f128)n, &overflow);
    }
    free(re);
    free(im);
    return overflow ? -1 : 0;
}

/* decode: z_j = (1/s) Re(sum_t m_t zeta^(5^j t)) via a length-n DFT of m_t zeta^t */
void orc_decode(uint32_t n, const double *mcoef, double scale, double *z)
{
    uint32_t N = n / 2, twon = 2 * n;
    f128 *re = malloc(sizeof(f128) * n), *im = malloc(sizeof(f128) * n);
    const f128 *c_, *s_;
    unit_roots(n, &c_, &s_);
    for (uint32_t t = 0; t < n; t++) {
        re[t] = (f128)mcoef[t] * half_c[t];
        im[t] = (f128)mcoef[t] * half_s[t];
    }
    qdft(re, im, n, +1);
    uint64_t f = 1;
    for (uint32_t j = 0; j < N; j++) {
        z[j] = (double)(re[(f - 1) / 2] / (f128)scale);
        f = f * 5 % twon;
    }
    free(re);
    free(im);
}

/* ------------------------------------------------------------------ */
/* RNS polynomials: [nl][n] residues, limb l modulo mod[pidx[l]]       */
/* ------------------------------------------------------------------ */

/* a small signed polynomial reduced into each listed prime */
void orc_reduce_small(const orc_params *p, const int64_t *x, const uint32_t *pidx, uint32_t nl, uint64_t *out)
{
    uint32_t n = p->n;
    for (uint32_t l = 0; l < nl; l++) {
        uint64_t q = p->mod[pidx[l]];
        for (uint32_t t = 0; t < n; t++) {
            int64_t v = x[t];
            uint64_t r = v >= 0 ? (uint64_t)v % q : (q - ((uint64_t)(-(v + 1)) + 1) % q) % q;
            out[(size_t)l * n + t] = r;
        }
    }
}

/* sigma_g: x^t -> x^(t g mod 2n), with x^n = -1 */
void orc_automorph(const orc_params *p, const uint32_t *pidx, uint32_t nl, uint32_t g, const uint64_t *in,
                   uint64_t *out)
{
    uint32_t n = p->n;
    for (uint32_t l = 0; l < nl; l++) {
        uint64_t q = p->mod[pidx[l]];
        const uint64_t *a = in + (size_t)l * n;
        uint64_t *b = out + (size_t)l * n;
        for (uint32_t t = 0; t < n; t++) {
            uint64_t e = ((uint64_t)t * g) % (2ull * n);
            if (e < n) b[e] = a[t];
            else b[e - n] = a[t] ? q - a[t] : 0;
        }
    }
}

/* index lists: Q_l = q_0..q_l ; QP_l = q_0..q_l, p_0..p_{k-1} */
static uint32_t qp_list(const orc_params *p, uint32_t level, uint32_t *pidx)
{
    uint32_t c = 0;
    for (uint32_t i = 0; i <= level; i++) pidx[c++] = i;
    for (uint32_t t = 0; t < p->k; t++) pidx[c++] = p->L + 1 + t;
    return c;
}

/* ------------------------------------------------------------------ */
/* keys, encryption, decryption                                         */
/* ------------------------------------------------------------------ */

/* purposes of the random streams */
enum { P_SECRET = 1, P_PK_A = 2, P_PK_E = 3, P_SWK_A = 4, P_SWK_E = 5, P_ENC_V = 6, P_ENC_E0 = 7, P_ENC_E1 = 8 };

void orc_keygen_secret(const orc_params *p, uint64_t seed, int64_t *s)
{
    orc_sample_ternary(seed, P_SECRET, 0, p->n, s);
}

/* pk = (-a s + e, a) over q_0..q_L, coefficient form, layout [2][L+1][n] */
void orc_keygen_pk(const orc_params *p, uint64_t seed, double sigma, const int64_t *s, uint64_t *pk)
{
    uint32_t n = p->n, nl = p->L + 1;
    uint32_t pidx[ORC_MAXP];
    for (uint32_t i = 0; i < nl; i++) pidx[i] = i;
    uint64_t *a = pk + (size_t)nl * n, *b = pk;
    orc_sample_uniform(p, seed, P_PK_A, 0, pidx, nl, a);
    int64_t *e = malloc(sizeof(int64_t) * n);
    orc_sample_gauss(seed, P_PK_E, 0, n, sigma, e);
    uint64_t *sr = malloc(sizeof(uint64_t) * n * nl), *er = malloc(sizeof(uint64_t) * n * nl);
    orc_reduce_small(p, s, pidx, nl, sr);
    orc_reduce_small(p, e, pidx, nl, er);
#pragma omp parallel for
    for (uint32_t l = 0; l < nl; l++) {
        uint64_t q = p->mod[l];
        size_t o = (size_t)l * n;
        orc_polymul(a + o, sr + o, b + o, n, q, p->psi[l]);
        for (uint32_t t = 0; t < n; t++) b[o + t] = addmod(submod(0, b[o + t], q), er[o + t], q);
    }
    free(e); free(sr); free(er);
}

/* Rotation (Galois) key for sigma_g, hybrid key switching, layout
 * [dnum][2][L+1+k][n] over all primes q_0..q_L, p_0..p_{k-1}:
 *   b_j = -a_j s + e_j + [P]_{q_i} sigma_g(s) [i in digit j]   (mod q_i)
 *   b_j = -a_j s + e_j                                          (mod p_t)
 * i.e. the gadget is the CRT idempotent of digit j times P. */
void orc_keygen_swk(const orc_params *p, uint64_t seed, double sigma, const int64_t *s, uint32_t g, uint64_t *swk)
{
    uint32_t n = p->n, nl = p->L + 1 + p->k;
    uint32_t pidx[ORC_MAXP];
    for (uint32_t i = 0; i < nl; i++) pidx[i] = i;
    uint64_t *sr = malloc(sizeof(uint64_t) * n * nl), *sg = malloc(sizeof(uint64_t) * n * nl);
    orc_reduce_small(p, s, pidx, nl, sr);
    orc_automorph(p, pidx, nl, g, sr, sg);
    int64_t *e = malloc(sizeof(int64_t) * n);
    for (uint32_t j = 0; j < p->dnum; j++) {
        uint64_t idx = ((uint64_t)g << 8) | j;
        uint64_t *b = swk + (size_t)j * 2 * nl * n, *a = b + (size_t)nl * n;
        orc_sample_uniform(p, seed, P_SWK_A, idx, pidx, nl, a);
        orc_sample_gauss(seed, P_SWK_E, idx, n, sigma, e);
        uint64_t *er = malloc(sizeof(uint64_t) * n * nl);
        orc_reduce_small(p, e, pidx, nl, er);
#pragma omp parallel for
        for (uint32_t l = 0; l < nl; l++) {
            uint64_t q = p->mod[l];
            size_t o = (size_t)l * n;
            orc_polymul(a + o, sr + o, b + o, n, q, p->psi[l]);
            uint64_t Pm = 1;
            for (uint32_t t = 0; t < p->k; t++) Pm = orc_mulmod(Pm, p->mod[p->L + 1 + t] % q, q);
            int in_digit = l <= p->L && l / p->alpha == j;
            for (uint32_t t = 0; t < n; t++) {
                uint64_t v = addmod(submod(0, b[o + t], q), er[o + t], q);
                if (in_digit) v = addmod(v, orc_mulmod(Pm, sg[o + t], q), q);
                b[o + t] = v;
            }
        }
        free(er);
    }
    free(sr); free(sg); free(e);
}

/* The same key restricted to the primes pidx[0..nl) (any subset of all
 * L+1+k): every limb of a key depends only on its own prime's stream words
 * (uniform draws at word 2 n i of the stream for prime i) and on the shared
 * secret and error polynomials, so the listed limbs equal those of
 * orc_keygen_swk; the others are left untouched.  Same layout
 * [dnum][2][L+1+k][n].  For tests that rotate only at low levels. */
void orc_keygen_swk_limbs(const orc_params *p, uint64_t seed, double sigma, const int64_t *s, uint32_t g,
                          const uint32_t *pidx, uint32_t nl, uint64_t *swk)
{
    uint32_t n = p->n, NLK = p->L + 1 + p->k;
    int64_t *e = malloc(sizeof(int64_t) * n);
    for (uint32_t j = 0; j < p->dnum; j++) {
        uint64_t idx = ((uint64_t)g << 8) | j;
        orc_sample_gauss(seed, P_SWK_E, idx, n, sigma, e);
#pragma omp parallel for
        for (uint32_t l = 0; l < nl; l++) {
            uint32_t pi = pidx[l];
            uint64_t q = p->mod[pi];
            uint64_t *b = swk + ((size_t)j * 2 * NLK + pi) * n, *a = b + (size_t)NLK * n;
            uint64_t *w = malloc(sizeof(uint64_t) * 2 * n), *sr = malloc(sizeof(uint64_t) * n);
            uint64_t *sg = malloc(sizeof(uint64_t) * n), *er = malloc(sizeof(uint64_t) * n);
            orc_stream_u64(seed, P_SWK_A, idx, 2ull * pi * n, 2ull * n, w);
            for (uint32_t t = 0; t < n; t++) {
                u128 v = ((u128)w[2 * t] << 64) | w[2 * t + 1];
                a[t] = (uint64_t)(v % q);
            }
            orc_reduce_small(p, s, &pi, 1, sr);
            orc_automorph(p, &pi, 1, g, sr, sg);
            orc_reduce_small(p, e, &pi, 1, er);
            orc_polymul(a, sr, b, n, q, p->psi[pi]);
            uint64_t Pm = 1;
            for (uint32_t t = 0; t < p->k; t++) Pm = orc_mulmod(Pm, p->mod[p->L + 1 + t] % q, q);
            int in_digit = pi <= p->L && pi / p->alpha == j;
            for (uint32_t t = 0; t < n; t++) {
                uint64_t v = addmod(submod(0, b[t], q), er[t], q);
                if (in_digit) v = addmod(v, orc_mulmod(Pm, sg[t], q), q);
                b[t] = v;
            }
            free(w); free(sr); free(sg); free(er);
        }
    }
    free(e);
}

/* Relinearization key: the key-switching key of orc_keygen_swk with s^2 in
 * place of sigma_g(s) (the target of the d2 s^2 term of a product), random
 * streams indexed by the digit alone (Galois elements are odd, so the index
 * (g << 8) | j of a rotation key never takes these values). */
void orc_keygen_relin(const orc_params *p, uint64_t seed, double sigma, const int64_t *s, uint64_t *rlk)
{
    uint32_t n = p->n, nl = p->L + 1 + p->k;
    uint32_t pidx[ORC_MAXP];
    for (uint32_t i = 0; i < nl; i++) pidx[i] = i;
    uint64_t *sr = malloc(sizeof(uint64_t) * n * nl), *s2 = malloc(sizeof(uint64_t) * n * nl);
    orc_reduce_small(p, s, pidx, nl, sr);
#pragma omp parallel for
    for (uint32_t l = 0; l < nl; l++)
        orc_polymul(sr + (size_t)l * n, sr + (size_t)l * n, s2 + (size_t)l * n, n, p->mod[l], p->psi[l]);
    int64_t *e = malloc(sizeof(int64_t) * n);
    for (uint32_t j = 0; j < p->dnum; j++) {
        uint64_t *b = rlk + (size_t)j * 2 * nl * n, *a = b + (size_t)nl * n;
        orc_sample_uniform(p, seed, P_SWK_A, j, pidx, nl, a);
        orc_sample_gauss(seed, P_SWK_E, j, n, sigma, e);
        uint64_t *er = malloc(sizeof(uint64_t) * n * nl);
        orc_reduce_small(p, e, pidx, nl, er);
#pragma omp parallel for
        for (uint32_t l = 0; l < nl; l++) {
            uint64_t q = p->mod[l];
            size_t o = (size_t)l * n;
            orc_polymul(a + o, sr + o, b + o, n, q, p->psi[l]);
            uint64_t Pm = 1;
            for (uint32_t t = 0; t < p->k; t++) Pm = orc_mulmod(Pm, p->mod[p->L + 1 + t] % q, q);
            int in_digit = l <= p->L && l / p->alpha == j;
            for (uint32_t t = 0; t < n; t++) {
                uint64_t v = addmod(submod(0, b[o + t], q), er[o + t], q);
                if (in_digit) v = addmod(v, orc_mulmod(Pm, s2[o + t], q), q);
                b[o + t] = v;
            }
        }
        free(er);
    }
    free(sr); free(s2); free(e);
}

/* ct = (v b + e0 + m, v a + e1) restricted to q_0..q_level; m is [level+1][n] */
void orc_encrypt(const orc_params *p, const uint64_t *pk, double sigma, const uint64_t *m, uint32_t level,
                 uint64_t seed, uint64_t index, uint64_t *ct)
{
    uint32_t n = p->n, nl = level + 1, NL = p->L + 1;
    uint32_t pidx[ORC_MAXP];
    for (uint32_t i = 0; i < nl; i++) pidx[i] = i;
    int64_t *v = malloc(sizeof(int64_t) * n), *e0 = malloc(sizeof(int64_t) * n), *e1 = malloc(sizeof(int64_t) * n);
    orc_sample_ternary(seed, P_ENC_V, index, n, v);
    orc_sample_gauss(seed, P_ENC_E0, index, n, sigma, e0);
    orc_sample_gauss(seed, P_ENC_E1, index, n, sigma, e1);
    uint64_t *vr = malloc(sizeof(uint64_t) * n * nl), *e0r = malloc(sizeof(uint64_t) * n * nl),
             *e1r = malloc(sizeof(uint64_t) * n * nl);
    orc_reduce_small(p, v, pidx, nl, vr);
    orc_reduce_small(p, e0, pidx, nl, e0r);
    orc_reduce_small(p, e1, pidx, nl, e1r);
#pragma omp parallel for
    for (uint32_t l = 0; l < nl; l++) {
        uint64_t q = p->mod[l];
        size_t o = (size_t)l * n;
        uint64_t *c0 = ct + o, *c1 = ct + (size_t)nl * n + o;
        orc_polymul(vr + o, pk + o, c0, n, q, p->psi[l]);
        orc_polymul(vr + o, pk + (size_t)NL * n + o, c1, n, q, p->psi[l]);
        for (uint32_t t = 0; t < n; t++) {
            c0[t] = addmod(addmod(c0[t], e0r[o + t], q), m[o + t], q);
            c1[t] = addmod(c1[t], e1r[o + t], q);
        }
    }
    free(v); free(e0); free(e1); free(vr); free(e0r); free(e1r);
}

/* m = c0 + c1 s mod q_0..q_level */
void orc_decrypt(const orc_params *p, const int64_t *s, const uint64_t *ct, uint32_t level, uint64_t *m)
{
    uint32_t n = p->n, nl = level + 1;
    uint32_t pidx[ORC_MAXP];
    for (uint32_t i = 0; i < nl; i++) pidx[i] = i;
    uint64_t *sr = malloc(sizeof(uint64_t) * n * nl);
    orc_reduce_small(p, s, pidx, nl, sr);
#pragma omp parallel for
    for (uint32_t l = 0; l < nl; l++) {
        uint64_t q = p->mod[l];
        size_t o = (size_t)l * n;
        orc_polymul(ct + (size_t)nl * n + o, sr + o, m + o, n, q, p->psi[l]);
        for (uint32_t t = 0; t < n; t++) m[o + t] = addmod(m[o + t], ct[o + t], q);
    }
    free(sr);
}

/* ------------------------------------------------------------------ */
/* hybrid key switching                                                 */
/* ------------------------------------------------------------------ */

/* ModUp of digit j of x (x over q_0..q_level, coefficient form) onto
 * QP_level = q_0..q_level, p_0..p_{k-1} by fast base conversion:
 *   y_t = sum_{i in D} [x_i (D/q_i)^-1]_{q_i} (D/q_i mod t)  (mod t)
 * with D the product of the digit's primes at this level; residues are used
 * as they are, in [0, q_i), without centering or correction. */
void orc_modup(const orc_params *p, uint32_t level, uint32_t j, const uint64_t *x, uint64_t *out)
{
    uint32_t n = p->n;
    uint32_t pidx[ORC_MAXP];
    uint32_t nout = qp_list(p, level, pidx);
    uint32_t lo = j * p->alpha, hi = (j + 1) * p->alpha;
    if (hi > level + 1) hi = level + 1;
#pragma omp parallel for
    for (uint32_t o = 0; o < nout; o++) {
        uint32_t ti = pidx[o];
        uint64_t t = p->mod[ti];
        uint64_t *y = out + (size_t)o * n;
        if (ti >= lo && ti < hi) { memcpy(y, x + (size_t)ti * n, sizeof(uint64_t) * n); continue; }
        memset(y, 0, sizeof(uint64_t) * n);
        for (uint32_t i = lo; i < hi; i++) {
            uint64_t qi = p->mod[i];
            uint64_t dhat_qi = 1, dhat_t = 1;
            for (uint32_t i2 = lo; i2 < hi; i2++)
                if (i2 != i) {
                    dhat_qi = orc_mulmod(dhat_qi, p->mod[i2] % qi, qi);
                    dhat_t = orc_mulmod(dhat_t, p->mod[i2] % t, t);
                }
            uint64_t inv = orc_invmod(dhat_qi, qi);
            const uint64_t *xi = x + (size_t)i * n;
            for (uint32_t c = 0; c < n; c++) {
                uint64_t a = orc_mulmod(xi[c], inv, qi);
                y[c] = addmod(y[c], orc_mulmod(a % t, dhat_t, t), t);
            }
        }
    }
}

/* ModDown: x over QP_level -> (x - Conv_{P->Q}(x_P)) * P^-1 over Q_level,
 *   y_i = sum_t [x_t (P/p_t)^-1]_{p_t} (P/p_t mod q_i)  (mod q_i)
 * (fast base conversion without correction). */
void orc_moddown(const orc_params *p, uint32_t level, const uint64_t *x, uint64_t *out)
{
    uint32_t n = p->n, k = p->k;
#pragma omp parallel for
    for (uint32_t i = 0; i <= level; i++) {
        uint64_t qi = p->mod[i];
        uint64_t *y = malloc(sizeof(uint64_t) * n);
        memset(y, 0, sizeof(uint64_t) * n);
        for (uint32_t t = 0; t < k; t++) {
            uint64_t pt = p->mod[p->L + 1 + t];
            uint64_t phat_pt = 1, phat_qi = 1;
            for (uint32_t t2 = 0; t2 < k; t2++)
                if (t2 != t) {
                    uint64_t p2 = p->mod[p->L + 1 + t2];
                    phat_pt = orc_mulmod(phat_pt, p2 % pt, pt);
                    phat_qi = orc_mulmod(phat_qi, p2 % qi, qi);
                }
            uint64_t inv = orc_invmod(phat_pt, pt);
            const uint64_t *xt = x + (size_t)(level + 1 + t) * n;
            for (uint32_t c = 0; c < n; c++) {
                uint64_t a = orc_mulmod(xt[c], inv, pt);
                y[c] = addmod(y[c], orc_mulmod(a % qi, phat_qi, qi), qi);
            }
        }
        uint64_t Pinv = 1;
        for (uint32_t t = 0; t < k; t++) Pinv = orc_mulmod(Pinv, p->mod[p->L + 1 + t] % qi, qi);
        Pinv = orc_invmod(Pinv, qi);
        for (uint32_t c = 0; c < n; c++) out[(size_t)i * n + c] = orc_mulmod(submod(x[(size_t)i * n + c], y[c], qi), Pinv, qi);
        free(y);
    }
}

/* Hoisted rotations of one ciphertext (coefficient form, [2][level+1][n]).
 * ModUp happens once, before any automorphism; for each Galois element g:
 *   D_j <- sigma_g(ModUp_j(c1)),  (e0, e1) = sum_j D_j * swk_{g,j}  over QP,
 *   out = (sigma_g(c0) + ModDown(e0), ModDown(e1)).
 * swk_ntt[r] is the key for gs[r] with every limb already in NTT form
 * (orc_ntt), layout [dnum][2][L+1+k][n]; outs[r] receives [2][level+1][n]. */
void orc_rotate_hoisted(const orc_params *p, uint32_t level, const uint64_t *ct, uint32_t nrot, const uint32_t *gs,
                        const uint64_t *const *swk_ntt, uint64_t *const *outs)
{
    uint32_t n = p->n, nq = level + 1, NLK = p->L + 1 + p->k;
    uint32_t beta = (nq + p->alpha - 1) / p->alpha;
    uint32_t pidx[ORC_MAXP];
    uint32_t nqp = qp_list(p, level, pidx);
    const uint64_t *c0 = ct, *c1 = ct + (size_t)nq * n;
    uint64_t *D = malloc(sizeof(uint64_t) * beta * nqp * n);
    for (uint32_t j = 0; j < beta; j++) orc_modup(p, level, j, c1, D + (size_t)j * nqp * n);
    uint64_t *e = malloc(sizeof(uint64_t) * 2 * nqp * n);
    for (uint32_t r = 0; r < nrot; r++) {
        uint32_t g = gs[r];
#pragma omp parallel for
        for (uint32_t o = 0; o < nqp; o++) {
            uint32_t pi = pidx[o];
            uint64_t q = p->mod[pi];
            uint64_t *acc0 = calloc(n, sizeof(uint64_t)), *acc1 = calloc(n, sizeof(uint64_t));
            uint64_t *d = malloc(sizeof(uint64_t) * n);
            for (uint32_t j = 0; j < beta; j++) {
                orc_automorph(p, &pi, 1, g, D + ((size_t)j * nqp + o) * n, d);
                orc_ntt(d, n, q, p->psi[pi]);
                const uint64_t *kb = swk_ntt[r] + ((size_t)j * 2 * NLK + pi) * n;
                const uint64_t *ka = swk_ntt[r] + ((size_t)j * 2 * NLK + NLK + pi) * n;
                for (uint32_t c = 0; c < n; c++) {
                    acc0[c] = addmod(acc0[c], orc_mulmod(d[c], kb[c], q), q);
                    acc1[c] = addmod(acc1[c], orc_mulmod(d[c], ka[c], q), q);
                }
            }
            orc_intt(acc0, n, q, p->psi[pi]);
            orc_intt(acc1, n, q, p->psi[pi]);
            memcpy(e + (size_t)o * n, acc0, sizeof(uint64_t) * n);
            memcpy(e + (size_t)(nqp + o) * n, acc1, sizeof(uint64_t) * n);
            free(acc0); free(acc1); free(d);
        }
        uint64_t *out = outs[r];
        orc_moddown(p, level, e, out);
        orc_moddown(p, level, e + (size_t)nqp * n, out + (size_t)nq * n);
        uint64_t *rc0 = malloc(sizeof(uint64_t) * nq * n);
        orc_automorph(p, pidx, nq, g, c0, rc0);
        for (uint32_t i = 0; i < nq; i++)
            for (uint32_t c = 0; c < n; c++)
                out[(size_t)i * n + c] = addmod(out[(size_t)i * n + c], rc0[(size_t)i * n + c], p->mod[i]);
        free(rc0);
    }
    free(D);
    free(e);
}

/* The key-switch products of hoisted rotations without their ModDown:
 * for each g, e_out[r] (layout [2][level+1+k][n], coefficient form over
 * q_0..q_level, p_0..p_{k-1}) = sum_j sigma_g(ModUp_j(c1)) * swk_{g,j}.
 * ModDown of e_out[r], plus sigma_g(c0), is exactly orc_rotate_hoisted. */
void orc_keyswitch_raw(const orc_params *p, uint32_t level, const uint64_t *ct, uint32_t nrot, const uint32_t *gs,
                       const uint64_t *const *swk_ntt, uint64_t *const *e_out)
{
    uint32_t n = p->n, nq = level + 1, NLK = p->L + 1 + p->k;
    uint32_t beta = (nq + p->alpha - 1) / p->alpha;
    uint32_t pidx[ORC_MAXP];
    uint32_t nqp = qp_list(p, level, pidx);
    const uint64_t *c1 = ct + (size_t)nq * n;
    uint64_t *D = malloc(sizeof(uint64_t) * beta * nqp * n);
    for (uint32_t j = 0; j < beta; j++) orc_modup(p, level, j, c1, D + (size_t)j * nqp * n);
    for (uint32_t r = 0; r < nrot; r++) {
        uint32_t g = gs[r];
        uint64_t *e = e_out[r];
#pragma omp parallel for
        for (uint32_t o = 0; o < nqp; o++) {
            uint32_t pi = pidx[o];
            uint64_t q = p->mod[pi];
            uint64_t *acc0 = calloc(n, sizeof(uint64_t)), *acc1 = calloc(n, sizeof(uint64_t));
            uint64_t *d = malloc(sizeof(uint64_t) * n);
            for (uint32_t j = 0; j < beta; j++) {
                orc_automorph(p, &pi, 1, g, D + ((size_t)j * nqp + o) * n, d);
                orc_ntt(d, n, q, p->psi[pi]);
                const uint64_t *kb = swk_ntt[r] + ((size_t)j * 2 * NLK + pi) * n;
                const uint64_t *ka = swk_ntt[r] + ((size_t)j * 2 * NLK + NLK + pi) * n;
                for (uint32_t c = 0; c < n; c++) {
                    acc0[c] = addmod(acc0[c], orc_mulmod(d[c], kb[c], q), q);
                    acc1[c] = addmod(acc1[c], orc_mulmod(d[c], ka[c], q), q);
                }
            }
            orc_intt(acc0, n, q, p->psi[pi]);
            orc_intt(acc1, n, q, p->psi[pi]);
            memcpy(e + (size_t)o * n, acc0, sizeof(uint64_t) * n);
            memcpy(e + (size_t)(nqp + o) * n, acc1, sizeof(uint64_t) * n);
            free(acc0); free(acc1); free(d);
        }
    }
    free(D);
}

/* out = a * b limb by limb (polynomial products), limb l modulo mod[pidx[l]] */
void orc_mul_limbs(const orc_params *p, const uint32_t *pidx, uint32_t nl, const uint64_t *a, const uint64_t *b,
                   uint64_t *out)
{
    uint32_t n = p->n;
#pragma omp parallel for
    for (uint32_t l = 0; l < nl; l++)
        orc_polymul(a + (size_t)l * n, b + (size_t)l * n, out + (size_t)l * n, n, p->mod[pidx[l]], p->psi[pidx[l]]);
}

/* out = a + b limb by limb, limb l modulo mod[pidx[l]] */
void orc_add_limbs(const orc_params *p, const uint32_t *pidx, uint32_t nl, const uint64_t *a, const uint64_t *b,
                   uint64_t *out)
{
    uint32_t n = p->n;
    for (uint32_t l = 0; l < nl; l++) {
        uint64_t q = p->mod[pidx[l]];
        for (uint32_t c = 0; c < n; c++) out[(size_t)l * n + c] = addmod(a[(size_t)l * n + c], b[(size_t)l * n + c], q);
    }
}

/* ------------------------------------------------------------------ */
/* plaintext products, additions, rescale                               */
/* ------------------------------------------------------------------ */

/* out = ct * pt (each polynomial of ct times pt), [2][level+1][n] */
void orc_mul_pt(const orc_params *p, uint32_t level, const uint64_t *ct, const uint64_t *pt, uint64_t *out)
{
    uint32_t n = p->n, nq = level + 1;
#pragma omp parallel for
    for (uint32_t w = 0; w < 2 * nq; w++) {
        uint32_t i = w % nq;
        orc_polymul(ct + (size_t)w * n, pt + (size_t)i * n, out + (size_t)w * n, n, p->mod[i], p->psi[i]);
    }
}

/* out = a + b (nl limbs over q_0..q_{nl-1}, nrep polynomials) */
void orc_add(const orc_params *p, uint32_t nl, uint32_t nrep, const uint64_t *a, const uint64_t *b, uint64_t *out)
{
    uint32_t n = p->n;
    for (uint32_t r = 0; r < nrep; r++)
        for (uint32_t i = 0; i < nl; i++) {
            uint64_t q = p->mod[i];
            size_t o = ((size_t)r * nl + i) * n;
            for (uint32_t c = 0; c < n; c++) out[o + c] = addmod(a[o + c], b[o + c], q);
        }
}

/* Rescale by the last prime q_l: r = c_l centered into [-(q_l-1)/2, (q_l-1)/2],
 * c'_i = (c_i - r) * q_l^-1 mod q_i for i < l.  in [2][l+1][n] -> out [2][l][n]. */
void orc_rescale(const orc_params *p, uint32_t level, const uint64_t *ct, uint64_t *out)
{
    uint32_t n = p->n, nq = level + 1;
    uint64_t ql = p->mod[level];
    for (uint32_t poly = 0; poly < 2; poly++) {
        const uint64_t *c = ct + (size_t)poly * nq * n;
        uint64_t *o = out + (size_t)poly * level * n;
        const uint64_t *last = c + (size_t)level * n;
        for (uint32_t i = 0; i < level; i++) {
            uint64_t qi = p->mod[i];
            uint64_t inv = orc_invmod(ql % qi, qi);
            for (uint32_t t = 0; t < n; t++) {
                uint64_t v = last[t];
                uint64_t r; /* centered residue, reduced mod q_i */
                if (v <= (ql - 1) / 2) r = v % qi;
                else r = submod(0, (ql - v) % qi, qi);
                o[(size_t)i * n + t] = orc_mulmod(submod(c[(size_t)i * n + t], r, qi), inv, qi);
            }
        }
    }
}

/* limb-wise NTT of nl limbs (used by callers to put keys in evaluation form) */
void orc_ntt_limbs(const orc_params *p, const uint32_t *pidx, uint32_t nl, uint64_t *a)
{
#pragma omp parallel for
    for (uint32_t l = 0; l < nl; l++) orc_ntt(a + (size_t)l * p->n, p->n, p->mod[pidx[l]], p->psi[pidx[l]]);
}
