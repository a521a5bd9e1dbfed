// hec_common.h -- internal declarations shared by the host code and the
// gfx950 kernels of the RNS-CKKS conv/pool library.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>
#include <stddef.h>

typedef uint64_t u64;
typedef uint32_t u32;

// Per-prime constants in device memory.
struct PrimeC {
    u64 q;
    u64 qinv_neg;  // -q^-1 mod 2^64 (Montgomery reduction)
    u64 r2;        // 2^128 mod q (into Montgomery form)
    u64 ninv;      // n^-1 mod q
    u64 ninv_sh;   // Shoup companion of ninv
    double qd, ninv_q;  // q and n^-1 / q as doubles (primes below 2^50: the exact double butterflies)
    double qinv_d;      // 1 / q rounded to the nearest double
    u32 fp;             // q < 2^50: the 2^16 transforms may run in doubles
    u32 pad_;
};

// Fast base conversion from `nin` limbs to `nout` limbs (ModUp of one digit,
// or the P -> Q conversion of ModDown):
//   a_i = [x_i * inv_hat_i]_{q_i},  y_o = sum_i a_i * (hat_i mod t_o)  (mod t_o)
// hat_m holds (hat_i mod t_o) * 2^64 mod t_o so that one Montgomery reduction
// of the 128-bit sum gives y_o directly.
#define HEC_MAX_BCONV_IN 16
#define HEC_MAX_LIMBS 64
struct BconvDesc {
    u32 nin, nout;
    u32 in_pos[HEC_MAX_BCONV_IN];   // limb positions of the inputs in the source buffer
    u32 in_prime[HEC_MAX_BCONV_IN];
    u64 inv_hat[HEC_MAX_BCONV_IN];
    u64 inv_hat_sh[HEC_MAX_BCONV_IN];
    u32 out_pos[HEC_MAX_LIMBS];     // limb positions of the outputs in the destination buffer
    u32 out_prime[HEC_MAX_LIMBS];
    u64 hat_m[HEC_MAX_BCONV_IN * HEC_MAX_LIMBS];  // [nin][nout]
};

// Per-level constants of rescale and ModDown.
struct LevelC {
    u64 qlinv[HEC_MAX_LIMBS];      // q_level^-1 mod q_i (i < level)
    u64 qlinv_sh[HEC_MAX_LIMBS];
    u64 pinv[HEC_MAX_LIMBS];       // P^-1 mod q_i
    u64 pinv_sh[HEC_MAX_LIMBS];
};

// Device tables of a context.
struct DevTables {
    u32 logn, n, nprimes;
    const PrimeC *pc;
    const u64 *tw, *tw_sh;    // psi^brv(k), [prime][n]
    const u64 *itw, *itw_sh;  // psi^-brv(k), [prime][n]
    const double2 *twf, *itwf;  // (w, w / q) as doubles for the primes below 2^50, [prime][n]
    // forward row-pass twists of the 2^16 transforms (n = 2^16 only, else null), [prime][row][col]
    // of the 256 x 256 view: psi^(col (1 + 2 brv8(row))), with Shoup companions, and as doubles
    const u64 *z, *z_sh;
    const double *zf;
    u32 fp_on;                  // the 2^16 transforms of those primes in doubles (a launch parameter)
};

// scratch array of the allocation-free rotation, per device
#define HEC_NOALLOC_SCRATCH_BYTES (128ull << 20)

// HEC_KS_BATCH: terms per launch of the kernels that sum key-switch or
// plaintext products (their carry-free 30-bit sums hold at most 16);
// HEC_ROT_BATCH: rotations per key-switch launch of a hoisted set and per
// batch of ModDowns (no sums across entries, so larger launches)
#define HEC_KS_BATCH 16
#define HEC_ROT_BATCH 32
struct KsBatch {
    const u64 *key[HEC_ROT_BATCH];  // [dnum][2][L+1+k][n], Montgomery form
    u64 *out[HEC_ROT_BATCH];        // [2][nqp][n]
    const u64 *D[HEC_ROT_BATCH];    // this entry's own hoisted digits (null: the launch's shared D)
    // c0 of the rotated ciphertext ([nq][n], NTT form): P * sigma_g(c0) is
    // added to the Q limbs of polynomial 0, so that the ModDown that follows
    // yields ModDown(e) + sigma_g(c0) exactly (null: nothing added)
    const u64 *c0[HEC_ROT_BATCH];
    u32 g[HEC_ROT_BATCH];
};

// Key-stationary key switch: rotation t of a launch (key[t], g[t]) applied to
// every input u < S with bit u of mask[t] set (inputs' hoisted digits at
// D + u * dstride), e_{t,u} at out[t] + u * estride ([2][nqp][n]).
struct KsMulti {
    const u64 *key[HEC_KS_BATCH];  // [dnum][2][L+1+k][n], Montgomery form
    u64 *out[HEC_KS_BATCH];
    u64 mask[HEC_KS_BATCH];
    u32 g[HEC_KS_BATCH];
};
#define HEC_MULTI_MAX_INPUTS 64

// Key switching fused with plaintext products, accumulated before ModDown.
// Term t is a rotation by g[t] of ciphertext ct[t] (key[t] == null when
// g[t] == 1; D[t] its ModUp, unused then) whose result is multiplied by
// pt[t][v] (null: no product) and added into output v.  Outputs are
// [2][nqp][n] over Q_l and P; the Q limbs carry P * (product), so that one
// ModDown of the accumulator gives the sum.
// Up to HEC_MAC_OUT outputs per launch (more than two: in groups handled by
// neighbouring workgroups, which share the key and digit reads through L2).
#define HEC_MAC_OUT 20
struct KsMacBatch {
    const u64 *key[HEC_KS_BATCH];              // [dnum][2][L+1+k][n], Montgomery form
    const u64 *D[HEC_KS_BATCH];                // [beta][nqp][n], ModUp of ct[t]'s c1 (NTT form)
    const u64 *ct[HEC_KS_BATCH];               // [2][nq][n] (NTT form)
    const u64 *pt[HEC_KS_BATCH][HEC_MAC_OUT];  // [nqp][n], Montgomery form
    u32 g[HEC_KS_BATCH];
    u64 *E[HEC_MAC_OUT];                       // [2][nqp][n], NTT form
};

// Weight plaintexts in basis-mask form: the plaintext of a term for an output
// is sum_b w_b * E_{tap,b} over the blocks b of a shard, E_{tap,b} the encoded
// mask of the term's tap restricted to block b and w_b a small integer; the
// product kernels read the basis polynomials of a term once and combine them
// with every output's weights in registers.  With E null the plaintext
// pointers point at plaintexts; with E set they point at the nb weights
// (int64_t, |w| < 2^31) of each (term, output).
#define HEC_BASIS_NB 2
struct BasisArg {
    const u64 *E;            // [taps][nb][nqp][n], NTT + Montgomery form
    u32 tap[HEC_KS_BATCH];   // tap of each term
    u32 nb, nqp;             // blocks per shard; limbs of a basis polynomial and stride of a weight row
};

// Plaintext products of several rotated ciphertexts summed into several
// outputs in one pass: out_v (+)= sum_t ct_t * pt[t][v] over the Q limbs.
#define HEC_MAC_TERMS 16
#define HEC_MAC_OUTS 8
struct MacBatch {
    const u64 *ct[HEC_MAC_TERMS];                // [2][nq][n], NTT form
    const u64 *pt[HEC_MAC_TERMS][HEC_MAC_OUTS];  // Q limbs first, NTT + Montgomery form (null: no product)
    u64 *out[HEC_MAC_OUTS];                      // [2][nq][n]
};

struct CombineBatch {
    u64 *out[HEC_ROT_BATCH];        // [2][nq][n]
    const u64 *e[HEC_ROT_BATCH];    // [2][nqp][n], Q limbs in NTT form
    const u64 *y[HEC_ROT_BATCH];    // [2][nq][n], NTT form
    const u64 *c0[HEC_ROT_BATCH];   // this entry's own c0 (null: the launch's shared c0)
    const u64 *add[HEC_ROT_BATCH][2];  // [nq][n] added to poly 0 / 1 of the entry as is (null: nothing)
    u32 g[HEC_ROT_BATCH];
};

// Launch parameters the autotuner (hec_tune.cpp) chooses among; every choice
// gives the same residues.  Process-wide; read when work is enqueued.
struct TuneParams {
    int ntt16_radix = 16;  // 2^16 transforms: 16 = two radix-16 register passes, 2 = radix-2 LDS tiles
    int ntt_tile = 4096;   // words per LDS tile of the radix-2 transforms (2048, 4096, 8192)
    int ntt_group = 0;     // at most this many limbs per transform launch (0: all in one)
    int ks_rot_batch = 32; // rotations per key-switch launch of a hoisted set (1..HEC_ROT_BATCH)
    int ks_amounts = 4;    // amounts per key-stationary launch over many inputs (1..HEC_KS_BATCH)
    int ntt_fp64 = 1;      // 2^16 transforms of primes below 2^50 with exact double butterflies (0: integers)
    int ntt_row_vals = 16; // values per lane of the 2^16 forward row pass (16: 256 lanes per tile, 8: 512)
    int ks_overlap = 0;    // hoisted rotation batches alternate between two streams (0: all on one)
};
TuneParams &hec_tune_params();

// ---- launchers (hec_kernels.hip) -----------------------------------------
// NTT / INTT of `nlimbs` limbs of `npolys` polynomials: limb l of poly p sits
// at base + p*poly_stride + l*n and uses prime pmap[l] (device array).
void hec_ntt_fwd(const DevTables &T, u64 *base, size_t poly_stride, int npolys, const u32 *pmap, int nlimbs,
                 hipStream_t st);
void hec_ntt_inv(const DevTables &T, u64 *base, size_t poly_stride, int npolys, const u32 *pmap, int nlimbs,
                 hipStream_t st);

enum EwOp { EW_ADD = 0, EW_SUB, EW_NEG, EW_MUL_MONT, EW_MAC_MONT, EW_TO_MONT, EW_FROM_MONT, EW_COPY, EW_ZERO,
            EW_DBL_SUB };
// out = op(a, b) over nlimbs x n per poly (EW_DBL_SUB: 2a - b) (poly strides given separately for out/a/b; b stride may be 0 to
// broadcast one polynomial over all polys).
void hec_ew(const DevTables &T, EwOp op, u64 *out, const u64 *a, const u64 *b, size_t so, size_t sa, size_t sb,
            int npolys, const u32 *pmap, int nlimbs, hipStream_t st);

// out[l][t] = x[t] mod pmap[l] for a signed small polynomial x[n].
void hec_reduce_i64(const DevTables &T, u64 *out, const int64_t *x, const u32 *pmap, int nlimbs, hipStream_t st);

// ChaCha20 samplers (stream named seed/purpose/index).
void hec_sample_uniform(const DevTables &T, u64 *out, u64 seed, u32 purpose, u64 index, const u32 *pmap,
                        int nlimbs, hipStream_t st);
void hec_sample_small(const DevTables &T, int64_t *out, u64 seed, u32 purpose, u64 index, int kind,
                      const u64 *gauss_T, hipStream_t st);

// Base conversion of npolys polynomials in groups of `group` that share a source: polynomial z uses
// descriptor d_desc[(z % group) * desc_stride], reads src + (z / group)*src_poly_stride and writes
// dst + z*dst_poly_stride; nout_max bounds the descriptors' nout and nin_max their nin.  copy_in also
// copies the input limbs to the same positions of the destination.
void hec_bconv(const DevTables &T, const BconvDesc *d_desc, int desc_stride, int group, int nout_max, const u64 *src,
               u64 *dst, size_t src_poly_stride, size_t dst_poly_stride, int npolys, int copy_in, hipStream_t st,
               int nin_max);

// pm, nq: [P * 2^64]_{q_i} of the Q limbs i < nq, for the entries with c0 set
void hec_ks_inner(const DevTables &T, const KsBatch &kb, int nrot, const u64 *D, int beta, int nqp, const u32 *pmap,
                  int NLK, hipStream_t st, const u64 *pm = nullptr, int nq = 0);
// the same products as hec_ks_inner for nrot <= HEC_KS_BATCH rotations x S <= HEC_MULTI_MAX_INPUTS inputs,
// each key read once for all inputs; false (nothing launched) for sizes out of range
bool hec_ks_inner_multi(const DevTables &T, const KsMulti &kb, int nrot, const u64 *D, size_t dstride, int S,
                        size_t estride, int beta, int nqp, const u32 *pmap, int NLK, hipStream_t st);

// E_v (+)= sum_t pt[t][v] * KS_t, KS_t = (sum_j sigma_g(D_j) key_j + P sigma_g(c0), sum_j sigma_g(D_j) key'_j)
// or P * (c0, c1) for g == 1, over the terms' own ciphertexts and ModUps (b.ct, b.D);
// pm[i] = P * 2^64 mod q_i; bit v of `first` set: output v is written instead of accumulated.
// Rotations by zero (g == 1) must precede the others; returns false (nothing launched) otherwise.
// ba (nullable): the plaintexts in basis-mask form.
bool hec_ks_mac(const DevTables &T, const KsMacBatch &b, int nterms, int nout, int beta, int nq, int nqp,
                const u32 *pmap, const u64 *pm, int NLK, int first, hipStream_t st, const BasisArg *ba = nullptr);

// The same products for S inputs at once (input u: D[t] + u ds, ct[t] + u cs, output E[0] + u es), each
// input with one output and the terms' keys and plaintexts (pt[t][0]) shared: the workgroups of the S
// inputs of one (limb, chunk) are neighbours, so a key or plaintext limb is read from HBM once for all of
// them.  Same residues as one hec_ks_mac per input.
struct ShardArg {
    u32 S;
    size_t ds, cs, es;
};
bool hec_ks_mac_shards(const DevTables &T, const KsMacBatch &b, int nterms, int beta, int nq, int nqp,
                       const u32 *pmap, const u64 *pm, int NLK, int first, const ShardArg &sh, hipStream_t st);

// the products of b (nterms <= HEC_MAC_TERMS, nout <= HEC_MAC_OUTS) summed in 128 bits and reduced once
// (the same residues as multiply-accumulating them one at a time); bit v of `first`: output v written
// false (nothing launched) for sizes out of range
bool hec_mac_terms(const DevTables &T, const MacBatch &b, int nterms, int nout, int nq, int first, hipStream_t st,
                   const BasisArg *ba = nullptr);

void hec_moddown_combine(const DevTables &T, const CombineBatch &cb, int nrot, const u64 *c0, int nq, int nqp,
                         const LevelC *lc, const u32 *pmap, hipStream_t st);

// Rescale of npolys polynomials at level l by q_l with its last two steps
// fused into the forward NTT (2N = 2^16 only): the column pass reads the
// dropped limb's coefficients (last, coefficient form, poly stride ls) and
// reduces their centered values mod each q_i, the row pass writes
// out_i = (c_i - NTT(r)_i) q_l^-1 (c and out with their poly strides); tmp
// ([npolys][l][n]) holds the column pass's output; pmap the identity map of
// the Q limbs.  Same residues as spread + NTT + finish.  Returns false
// (nothing launched) for another ring size.
struct RescaleFuse {
    const u64 *last;
    size_t ls;
    const u64 *c;
    size_t cs;
    u64 *out;
    size_t os;
    const LevelC *lc;
    u32 level;
};
// inverse NTT of nlimbs limbs of npolys polynomials read from src (poly stride
// src_stride) and written to dst (dst_stride); 2N = 2^16 only (false otherwise)
bool hec_ntt_inv_from(const DevTables &T, u64 *dst, size_t dst_stride, const u64 *src, size_t src_stride,
                      int npolys, const u32 *pmap, int nlimbs, hipStream_t st);
bool hec_ntt_fwd_rescale(const DevTables &T, u64 *tmp, int npolys, const u32 *pmap, const RescaleFuse &f,
                         hipStream_t st);
// ModDown tail of nrot <= HEC_ROT_BATCH entries fused into the forward NTT of
// their P -> Q conversions y ([2 nrot][nq][n], coefficient form; overwritten
// by the column pass): out_r = (e_r - NTT(y_r)) P^-1 + sigma_g(c0_r) (+ add),
// the residues of hec_ntt_fwd + hec_moddown_combine; 2N = 2^16 only (false,
// nothing launched, otherwise)
bool hec_ntt_fwd_moddown(const DevTables &T, u64 *y, int nrot, int nq, int nqp, const CombineBatch &cb,
                         const LevelC *lc, const u32 *pmap, hipStream_t st);
void hec_rescale_spread(const DevTables &T, const u64 *last_coef, u64 *tmp, size_t last_stride, size_t tmp_stride,
                        int npolys, u32 level, hipStream_t st);
void hec_rescale_finish(const DevTables &T, u64 *out, const u64 *c, const u64 *tmp, size_t so, size_t sc,
                        size_t st_, int npolys, u32 level, const LevelC *lc, hipStream_t st);

// swk/pk assembly: b = -a*s + e (+ pm * sigma_g(s) on limbs in [dlo, dhi); pm * tgt instead when tgt is
// given), then both b and a into Montgomery form.  sN is s in NTT form (plain), all primes; a, e, tgt in
// NTT form.
void hec_key_finish(const DevTables &T, u64 *b, u64 *a, const u64 *e, const u64 *sN, const u64 *tgt, const u64 *pm,
                    u32 g, u32 dlo, u32 dhi, int nlimbs, const u32 *pmap, hipStream_t st);

// per-limb constants (limb l = prime l) with Shoup companions
struct ScalarArg {
    u64 v[HEC_MAX_LIMBS];
    u64 vsh[HEC_MAX_LIMBS];
};
enum ScalarOp { SC_MUL = 0, SC_ADD, SC_MAC, SC_DBL_ADD };
// per limb l < nlimbs of npolys polynomials (in read with its own poly stride):
// SC_MUL out = in * v_l; SC_ADD out = in + v_l on even polys (the c0 of a ciphertext), in on odd ones;
// SC_MAC out (+)= in * v_l (first != 0: written); SC_DBL_ADD out = 2 in + v_l on even polys, 2 in on odd ones
void hec_scalar(const DevTables &T, ScalarOp op, u64 *out, const u64 *in, size_t out_poly_stride,
                size_t in_poly_stride, int npolys, int nlimbs, int first, const ScalarArg &sa, hipStream_t st);
// out = sum_j in_j * c_j over up to HEC_LIN_TERMS inputs, limbs l < nlimbs <= HEC_LIN_LIMBS of npolys
// polynomials (input j read with its own poly stride); c_j per limb in Montgomery form; the products
// summed in 128 bits and reduced once (the residues of multiply-accumulating them one at a time)
#define HEC_LIN_TERMS 8
#define HEC_LIN_LIMBS 32
struct LinArg {
    const u64 *in[HEC_LIN_TERMS];
    size_t ps[HEC_LIN_TERMS];
    u64 cm[HEC_LIN_TERMS][HEC_LIN_LIMBS];
};
bool hec_lincomb(const DevTables &T, u64 *out, size_t out_poly_stride, int npolys, int nlimbs, const LinArg &a,
                 int nterms, hipStream_t st);
// tensor products of cnt ciphertext pairs (a_i, b_i at a + 2i nq n, b + 2i nq n):
// t_i = [a0 b0][a1 b1][a0 b1 + a1 b0] at t + 3i nq n
void hec_tensor(const DevTables &T, u64 *t, const u64 *a, const u64 *b, int nq, int cnt, hipStream_t st);
// the same for nitems <= HEC_TENSOR_ITEMS separate batches of per pairs each
// (pair z = item z / per, index z % per in it), the results contiguous in t
#define HEC_TENSOR_ITEMS 16
struct TensorItems {
    const u64 *a[HEC_TENSOR_ITEMS];
    const u64 *b[HEC_TENSOR_ITEMS];
};
bool hec_tensor_items(const DevTables &T, u64 *t, const TensorItems &it, int nitems, int per, int nq, hipStream_t st);

// enc: c0 = v*pk0 + e0 + m, c1 = v*pk1 + e1 (pk in Montgomery form, the rest plain NTT form)
void hec_encrypt_finish(const DevTables &T, u64 *ct, const u64 *v, const u64 *e0, const u64 *e1, const u64 *m,
                        const u64 *pk, size_t pk_poly_stride, int nq, hipStream_t st);

// out[k] = in[perm_g(k)] (NTT-domain automorphism) for nlimbs x npolys
void hec_automorph_ntt(const DevTables &T, u64 *out, const u64 *in, size_t poly_stride, int npolys, int nlimbs,
                       u32 g, hipStream_t st);

// centered CRT of [nq][n] residues (coefficient form) into doubles; Mm[i][j] =
// prod_{k<j} q_k mod q_i in Montgomery form (row stride HEC_MAX_LIMBS), inv[i] =
// (prod_{k<i} q_k)^-1 mod q_i with its Shoup companion
void hec_crt_double(const DevTables &T, const u64 *res, double *out, int nq, const u64 *Mm, const u64 *inv,
                    const u64 *invsh, hipStream_t st);

// CKKS slot encoding of `count` vectors (z + i*zstride, nz values each) into signed coefficients
// m[count][n] (double-double FFT, rounding half away from zero); *flag != 0 afterwards if a
// coefficient reached 2^62.  work holds count * n double4.
void hec_encode(const double *z, size_t zstride, u32 nz, u32 count, double scale, const u32 *root,
                const double4 *tw, double4 *work, int64_t *m, int *flag, u32 logn, hipStream_t st);
// decoding of centered coefficients m[n] (doubles) into nz slot values; work holds n double2
void hec_decode(const double *m, double scale, const u32 *root, const double4 *tw, double2 *work, double *z,
                u32 nz, u32 logn, hipStream_t st);

// launch timing of one kernel by name (NULL stops); collect syncs the events
#define HEC_PROBE_MAX_READ 8
#define HEC_PROBE_MAX_WRITE 4
// nr (1..8) streams of `words` u64 at in read, nw (1..4) at out written
void hec_probe_stream(const u64 *in, u64 *out, size_t words, int nr, int nw, hipStream_t st);
void hec_prof_select(const char *name);
int hec_prof_collect(uint64_t *launches, uint64_t *units, double *ms);
uint64_t hec_prof_count(const char *name);

// dst[p][l] = src[p][l] for nl limbs (generic strided copy)
void hec_copy_limbs(u64 *dst, const u64 *src, size_t dst_poly_stride, size_t src_poly_stride, int npolys,
                    size_t limb_elems, hipStream_t st);
