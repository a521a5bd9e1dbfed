/*
 * hecnn.h -- C ABI of the MI355X (gfx950) library for homomorphic convolution
 * and average pooling on RNS-CKKS ciphertexts.
 *
 * Source of every operation: "High-Resolution Convolutional Neural Networks on
 * Homomorphically Encrypted Data via Sharding Ciphertexts" (Maloney et al.,
 * arXiv 2306.09189).
 *   - Background, "Homomorphic encryption": ciphertexts over
 *     Z_Q[x]/(x^n + 1), n = 2N, N real slots, levels, cyclic rotations;
 *   - Background, "Threat Model": the client encrypts and decrypts, the server
 *     evaluates with the weights in the clear;
 *   - Section 4 (packing, sharding, duplication/permutation), Section 4.1
 *     (convolution), Section 4.2 (average pooling), Section 4.3 (batch
 *     normalization folded into convolutions, linear and pool-linear layers,
 *     GELU) and the Appendix on polynomial approximation (Chebyshev basis).
 * The RNS-CKKS conventions the paper leaves to its library are fixed as
 * follows (and are what "bit-exact" refers to):
 *   - primes: for each requested size b, the first prime 2^b - j*2n + 1
 *     (j = 1, 2, ...) not yet taken, in the order q_0..q_L, p_0..p_{k-1};
 *   - hybrid key switching with dnum digits of alpha = ceil((L+1)/dnum)
 *     consecutive primes, CRT-idempotent gadget times P, fast base conversion
 *     on [0, q) residues without correction, ModDown by floor, ModUp before the
 *     automorphism (so rotate == rotate_hoisted bit for bit);
 *   - rotation by r > 0 moves slot j+r to slot j (Galois element 5^r mod 2n);
 *   - rescale rounds with the centered residue of the dropped limb;
 *   - randomness: ChaCha20 (RFC 8439) streams named (seed, purpose, index),
 *     fixed-length draws per coefficient; ternary secret, discrete Gaussian
 *     errors by table inversion;
 *   - encoding: canonical embedding on real slots, rounded half away from zero
 *     from a >= 100-bit evaluation of the exact value.
 *
 * Conventions of this interface:
 *   - every handle returned through an `out` pointer is owned by the caller and
 *     released with the matching *_free; inputs are borrowed, never retained;
 *   - on error nothing is returned (*out = NULL), the status code says why and
 *     hec_last_error() gives a message (thread-local, valid until the next
 *     call on that thread);
 *   - all device work of a context is ordered on the context's HIP stream;
 *     calls return after enqueueing, except the ones that hand data back to
 *     the host (decrypt, export), which synchronize the stream;
 *   - ciphertexts and plaintexts live in device memory in an internal form;
 *     export/import use the canonical comparison form: coefficient domain,
 *     layout [poly][limb][coeff], residues in [0, q_i).
 * Not thread-safe per context: one thread drives a context at a time.
 */
#ifndef HECNN_H
#define HECNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HEC_OK = 0,
    HEC_EINVAL = 1,  /* bad argument (sizes, null pointers, parameters)         */
    HEC_ENOMEM = 2,  /* device or host allocation failed                         */
    HEC_ELEVEL = 3,  /* level mismatch, or no level left to consume              */
    HEC_ESCALE = 4,  /* scale mismatch in an addition                            */
    HEC_ENOKEY = 5,  /* a rotation key the operation needs was not generated     */
    HEC_ELAYOUT = 6, /* the image layout cannot be planned for this operation    */
    HEC_EDEVICE = 7, /* HIP runtime error                                        */
    HEC_EBUSY = 8    /* context already in use                                   */
} hec_status;

typedef struct hec_ctx hec_ctx;
typedef struct hec_ct hec_ct;
typedef struct hec_pt hec_pt;
typedef struct hec_image hec_image;
typedef struct hec_conv_plan hec_conv_plan;
typedef struct hec_block hec_block;

/* RNS-CKKS parameters.  Ring degree n = 2^log_n (N = n/2 slots);
 * ciphertext primes q_0 (q0_bits) and q_1..q_L (q_bits each); k special
 * primes of p_bits; dnum key-switching digits; sigma the error standard
 * deviation; secret_dist 0 = uniform ternary (the only one supported).
 * log_scale is the default encoding scale 2^log_scale used by
 * he_image_encrypt.  Limits: 10 <= log_n <= 16, L + 1 + k <= 64,
 * 20 <= bits <= 60, dnum*alpha >= L+1. */
typedef struct {
    uint32_t log_n, L, q0_bits, q_bits, k, p_bits, dnum, log_scale;
    double sigma;
    uint32_t secret_dist;
} hec_params;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`, ordering all work on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  Builds the prime chain, the
 * NTT / base-conversion tables and uploads them. */
hec_status hec_ctx_create(const hec_params *params, int device, void *hip_stream, hec_ctx **out);
/* Waits for the context's stream and frees its device memory.  Every handle of
 * the context (ciphertexts, plaintexts, images, plans, blocks) must have been
 * freed before: they refer to the context's memory pool. */
void hec_ctx_destroy(hec_ctx *ctx);
const char *hec_last_error(void);

/* The primes of the context: q_0..q_L then p_0..p_{k-1} (L+1+k values). */
hec_status hec_ctx_primes(const hec_ctx *ctx, uint64_t *primes, size_t cap, size_t *count);
/* Number of slots N = n/2. */
uint32_t hec_ctx_slots(const hec_ctx *ctx);

/* ---- keys (Background: threat model; client side) ------------------------- */

/* Secret key, public key and the rotation keys for rot_steps[0..n_steps) from
 * one seed.  Each key depends only on (seed, its Galois element). */
hec_status ckks_keygen(hec_ctx *ctx, uint64_t seed, const int32_t *rot_steps, size_t n_steps);
/* More rotation keys from the seed given to ckks_keygen. */
hec_status ckks_gen_rotation_keys(hec_ctx *ctx, const int32_t *rot_steps, size_t n_steps);
/* Device bytes held by the rotation keys. */
size_t hec_ctx_key_bytes(const hec_ctx *ctx);
/* Key-switch inner products the context has computed so far (one per
 * rotation by a nonzero amount, whatever the evaluation mode). */
uint64_t hec_ctx_keyswitch_count(const hec_ctx *ctx);

/* ---- plaintexts / ciphertexts ---------------------------------------------- */

/* Encode nz <= N real slot values (the rest zero) at `level` and `scale`. */
hec_status ckks_encode(hec_ctx *ctx, const double *z, size_t nz, uint32_t level, double scale, hec_pt **out);
/* Public-key encryption of pt with randomness stream index 0 of `seed`. */
hec_status ckks_encrypt(hec_ctx *ctx, const hec_pt *pt, uint64_t seed, hec_ct **out);
/* Same with an explicit stream index. */
hec_status ckks_encrypt_idx(hec_ctx *ctx, const hec_pt *pt, uint64_t seed, uint64_t index, hec_ct **out);
/* Decrypt and decode the first nz <= N slots into z_out (host).  Synchronizes. */
hec_status ckks_decrypt(hec_ctx *ctx, const hec_ct *ct, double *z_out, size_t nz);

/* Left rotation by `step` slots (negative = right).  step % N == 0 copies. */
hec_status ckks_rotate(hec_ctx *ctx, const hec_ct *ct, int32_t step, hec_ct **out);
/* n rotations of one ciphertext sharing a single ModUp (the "rotations
 * computed once and cached" of Section 4.1).  outs[0..n) receive new handles. */
hec_status ckks_rotate_hoisted(hec_ctx *ctx, const hec_ct *ct, const int32_t *steps, size_t n, hec_ct **outs);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * rotation of ckks_rotate written into the caller's ciphertext `out` (created
 * beforehand at the input's level, e.g. by ckks_ct_import; not the input
 * itself), bit-identical to ckks_rotate.  Allocates, frees and synchronizes
 * nothing: its temporaries (c1 in coefficient form, the ModUp digits, the
 * key-switch product and the ModDown conversion: n * (3 (level+1) +
 * (beta + 2) (level+1+k)) words, beta = ceil((level+1)/alpha)) live in one
 * static device array of 128 MiB per GPU, held until the process ends (at
 * 2N = 2^16 with 8 special primes and 3 digits: 104 MiB at level 20, 120 MiB
 * at level 24); a rotation that needs more fails with HEC_EINVAL.  All calls on one GPU share that array: calls that overlap
 * on one GPU (several streams or contexts of the device, several threads)
 * race and must be ordered by the caller.  Errors: HEC_ELEVEL (out at another
 * level), HEC_ENOKEY, HEC_EINVAL; out keeps its contents on error. */
hec_status ckks_rotate_noalloc(hec_ctx *ctx, const hec_ct *in, int32_t step, hec_ct *out);
/* Divide by the last prime and drop it (level - 1, scale / q_level). */
hec_status ckks_rescale(hec_ctx *ctx, hec_ct *inout);
/* ct * pt (levels must match; scales multiply). */
hec_status ckks_mul_pt(hec_ctx *ctx, const hec_ct *ct, const hec_pt *pt, hec_ct **out);
/* a + b (levels and scales must match). */
hec_status ckks_add(hec_ctx *ctx, const hec_ct *a, const hec_ct *b, hec_ct **out);
/* ct + pt (pt at the ciphertext's level and scale: HEC_ELEVEL / HEC_ESCALE
 * otherwise; special-prime limbs of pt, if any, are ignored). */
hec_status ckks_add_pt(hec_ctx *ctx, const hec_ct *ct, const hec_pt *pt, hec_ct **out);
/* a - b (levels and scales must match). */
hec_status ckks_sub(hec_ctx *ctx, const hec_ct *a, const hec_ct *b, hec_ct **out);
/* Ciphertext product (the multiplications of the polynomial activation,
 * Section 4.3 "GELU" and Appendix "Polynomial Approximation"): tensor product
 * (a0 b0, a0 b1 + a1 b0, a1 b1), the s^2 part key-switched to s with the
 * relinearization key (hybrid key switching as for rotations; key target
 * s^2, random streams of the Galois element 0, generated from the keygen
 * seed on first use and kept by the context).  Levels must match; scale
 * a.scale * b.scale; not rescaled.  HEC_ENOKEY before ckks_keygen. */
hec_status ckks_mul(hec_ctx *ctx, const hec_ct *a, const hec_ct *b, hec_ct **out);
/* ct * value in every slot: value encoded at pscale as the constant polynomial
 * round_half_away(value * pscale) (the exact product of the two doubles; HEC_EINVAL
 * at or above 2^62); scale ct.scale * pscale, not rescaled. */
hec_status ckks_mul_const(hec_ctx *ctx, const hec_ct *ct, double value, double pscale, hec_ct **out);
/* ct + value in every slot, encoded the same way at the ciphertext's scale. */
hec_status ckks_add_const(hec_ctx *ctx, const hec_ct *ct, double value, hec_ct **out);
/* The first level+1 limbs of ct (level <= ct's level; scale kept). */
hec_status ckks_drop(hec_ctx *ctx, const hec_ct *ct, uint32_t level, hec_ct **out);
/* Level and scale of a ciphertext. */
hec_status ckks_ct_info(const hec_ct *ct, uint32_t *level, double *scale);

/* Canonical export: coeff receives [2][level+1][n] u64 (host).  Synchronizes. */
hec_status ckks_ct_export(hec_ctx *ctx, const hec_ct *ct, uint64_t *coeff, uint32_t *level, double *scale);
hec_status ckks_ct_import(hec_ctx *ctx, const uint64_t *coeff, uint32_t level, double scale, hec_ct **out);
/* Plaintexts as data: [level+1][n] residues, coefficient domain. */
hec_status ckks_pt_export(hec_ctx *ctx, const hec_pt *pt, uint64_t *coeff, uint32_t *level, double *scale);
hec_status ckks_pt_import(hec_ctx *ctx, const uint64_t *coeff, uint32_t level, double scale, hec_pt **out);
/* Signed integer coefficients of an encoding (before reduction into limbs). */
hec_status ckks_encode_coeffs(hec_ctx *ctx, const double *z, size_t nz, double scale, int64_t *m_out);

/* ---- images (Section 4: packing, sharding, duplication, permutation) ------ */

/* Pack x [C][H][W] (row-major channels, channel-major; zero padding of the
 * side to a power of two; image shards when m^2 C > N, consecutive d-fold
 * copies when the image underfills a shard), encode at scale 2^log_scale and
 * encrypt every shard at `level` with stream (seed, index = shard). */
hec_status he_image_encrypt(hec_ctx *ctx, const double *x, uint32_t C, uint32_t H, uint32_t W, uint32_t level,
                            uint64_t seed, hec_image **out);
/* Decrypt into x_out [C][H][W] in logical channel order.  Synchronizes. */
hec_status he_image_decrypt(hec_ctx *ctx, const hec_image *img, double *x_out);
/* Geometry: channels, real side, padded side, number of shards. */
hec_status he_image_info(const hec_image *img, uint32_t *C, uint32_t *H, uint32_t *W, uint32_t *mp,
                         uint32_t *n_shards);
/* Block map of shard u: lam[b] = logical channel of block b (-1 = empty),
 * N / (mp*mp) entries. */
hec_status he_image_block_map(const hec_image *img, uint32_t u, int32_t *lam, size_t cap);
/* Borrowed handle of shard u (valid while img lives). */
const hec_ct *he_image_shard(const hec_image *img, uint32_t u);
/* Channel shards (Section 4, channel side above sqrt(N)): shard u holds rows
 * part*R .. part*R+R-1 (R = N/mp) of logical channel `channel`.  Fails with
 * HEC_ELAYOUT on an image-sharded image (use he_image_block_map there). */
hec_status he_image_channel_shard(const hec_image *img, uint32_t u, int32_t *channel, int32_t *part);

/* Homomorphic conv2d (cross-correlation, zero padding `pad`, stride 1 or 2)
 * of an image-sharded input with weights w [Co][C][kh][kw] (PyTorch layout,
 * host doubles), Section 4.1: partial convolutions over hoisted rotations of
 * every input shard, fused weight x shift-mask plaintexts, one rescale per
 * output shard; stride 2 = stride-1 convolution + the downsampling of
 * Section 4.2.  w holds Co x C x kh x kw doubles, C the input image's channel
 * count (he_image_info).  bias (nullable): Co doubles, the per-channel shift
 * of an inference batch norm folded into the convolution (Section 4.3,
 * "Batch Normalization"), added to the output as he_image_add_bias does (one
 * plaintext per output shard at the output's level and scale).  Consumes one
 * level (three for stride 2 with the two-level downsample). */
hec_status he_conv2d_sharded(hec_ctx *ctx, const hec_image *in, const double *w, uint32_t Co, uint32_t kh,
                             uint32_t kw, uint32_t stride, uint32_t pad, const double *bias, hec_image **out);
/* The same split in two: plan once (weights encoded and kept in device memory
 * for the input's layout and level), then run on any image of that layout and
 * level.  Run is what a server repeats per request. */
hec_status he_conv2d_plan_create(hec_ctx *ctx, const hec_image *like, const double *w, uint32_t Co, uint32_t kh,
                                 uint32_t kw, uint32_t stride, uint32_t pad, hec_conv_plan **out);
/* With flags = HEC_PLAN_Q_ONLY the weight plaintexts are kept over Q_l only
 * (21 instead of 29 limbs at level 20 with 8 special primes): such a plan
 * runs in modes 0, 1 and 4, whose products follow complete rotations
 * (he_conv2d_plan_set_mode returns HEC_EINVAL for 2 and 3).  For layers whose plaintexts would not fit in HBM otherwise, e.g.
 * the 112x112x64 layer's 18432 plaintexts (267 GiB over Q and P, 193 GiB
 * over Q).  Unknown flag bits: HEC_EINVAL. */
#define HEC_PLAN_Q_ONLY 1u
/* With flags = HEC_PLAN_BASIS | HEC_PLAN_BASIS_SCALE(s), 1 <= s <= 50, the
 * weight plaintexts are kept in basis-mask form (Section 4.1: the plaintext
 * of a tap is, block by block, a kernel weight times the tap's mask, and the
 * masks are combined with the weights outside the encryption): per tap and
 * block b of a shard the mask restricted to b, encoded at 2^s over Q_l and P
 * (E_b), and per product the integers w^_b = round_half_away(w_b q_l / 2^s);
 * the plaintext is sum_b w^_b E_b, formed inside the product kernels.  Memory
 * taps x blocks x limbs instead of one plaintext per product (the
 * 112x112x64 layer: 261 MiB instead of 267 GiB), at the price of the
 * rounding of w^_b (2^(s-1) / q_l absolute per weight) and of E_b (relative
 * 2^-s).  Needs an image-sharded input with at most 2 blocks per shard
 * (HEC_ELAYOUT otherwise), |w^_b| < 2^31 and primes of at least 37 bits
 * (HEC_EINVAL otherwise); runs in modes 0, 1, 2 and 4 (he_conv2d_plan_set_mode
 * returns HEC_EINVAL for 3); excludes HEC_PLAN_Q_ONLY (HEC_EINVAL). */
#define HEC_PLAN_BASIS 2u
#define HEC_PLAN_BASIS_SCALE(s) ((uint32_t)(s) << 8)
hec_status he_conv2d_plan_create_ex(hec_ctx *ctx, const hec_image *like, const double *w, uint32_t Co, uint32_t kh,
                                    uint32_t kw, uint32_t stride, uint32_t pad, uint32_t flags, hec_conv_plan **out);
hec_status he_conv2d_plan_run(hec_ctx *ctx, const hec_conv_plan *plan, const hec_image *in, hec_image **out);
/* Execution mode of plan runs: 0 = batched (hoisted ModUp, rotations of a
 * shard batched per launch), 1 = plain (every rotation its own ModUp and
 * launch chain); both give identical ciphertexts.  2 = lazy ModDown (an
 * optimisation the paper does not describe: the key-switch products of all
 * rotations are multiplied by their weights and summed over Q_l and P, then
 * one ModDown per output shard); it rounds differently, so its ciphertexts
 * differ from modes 0/1 while decrypting to the same values within the same
 * error bound.  3 = baby-step / giant-step with double hoisting (also beyond
 * the paper): every rotation amount is a block offset (baby) plus a tap
 * offset (giant), pt * rot_{b+g}(ct) = rot_g(rot_{-g}(pt) * rot_b(ct)); the
 * weights rotated back by their giant step multiply the hoisted baby
 * rotations of each input (lazy ModDown per (giant, output) sum), and each
 * output sums its giant rotations of those sums with one more lazy ModDown --
 * babies + giants x outputs key switches instead of one per amount.  Its
 * plaintexts are encoded on the first switch to mode 3.  4 = key-stationary
 * batched: the ciphertexts of modes 0/1, with the rotations of all input
 * shards taken together amount by amount (Section 4.1, "With Image Shards":
 * every output shard sums over all input shards, which all rotate by the same
 * amounts), so each rotation key is read once per group of up to 64 shards
 * instead of once per shard, and the ModDowns of a batch of amounts x shards
 * share their launches.  Modes 2 and 3 also take the stride-2 downsampling
 * lazily (he_avgpool_ex mode 2), mode 4 key-stationary (he_avgpool_ex mode
 * 4).  Returns HEC_EINVAL for any other mode. */
hec_status he_conv2d_plan_set_mode(hec_conv_plan *plan, int mode);
/* Form of a stride-2 plan's downsampling step (Section 4.1, strided
 * convolution: the stride-1 convolution followed by the downsampling of the
 * pooling) independently of how the convolution itself runs: -1 = the plan
 * mode's own form (the default), or one of he_avgpool_ex's modes 0
 * (complete rotations), 2 (lazy ModDown) and 4 (key-stationary).  A server's
 * stem layer, for example, convolves key-stationary over Q-only plaintexts
 * and downsamples lazily.  HEC_EINVAL for other values or for a stride-1
 * plan. */
hec_status he_conv2d_plan_set_downsample_mode(hec_conv_plan *plan, int mode);
/* Rotation steps a plan (or an avgpool of `like`) needs keys for. */
hec_status he_conv2d_plan_steps(const hec_conv_plan *plan, int32_t *steps, size_t cap, size_t *count);
hec_status he_avgpool_steps(hec_ctx *ctx, const hec_image *like, int32_t *steps, size_t cap, size_t *count);
void he_conv2d_plan_free(hec_conv_plan *plan);

/* 2x2 average pooling, Section 4.2: downsample (2x2 window sums, horizontal
 * and vertical reduction with masks), consolidate groups of four shards,
 * duplicate when at most two shards were downsampled.  window must be 2.
 * Consumes two levels, or one when only one is left (reductions fused). */
hec_status he_avgpool(hec_ctx *ctx, const hec_image *in, uint32_t window, hec_image **out);
/* The same with an evaluation mode: 0 = as he_avgpool (every rotation of the
 * reductions key-switched and ModDown'd on its own); 2 = lazy ModDown (the
 * masked rotation sums of the reductions multiply the key-switch products
 * over Q_l and P and take one ModDown per sum -- an optimisation the paper
 * does not describe; other ciphertext bits, same values within the same
 * bound); 3 = as 2, except that masked sums of at least 32 rotations are
 * evaluated by baby and giant steps (amount = (i mod G) + (i - i mod G) in
 * units of the stage's shift, G = ceil(sqrt(count)); masks rotated back by the
 * giant step), also beyond the paper; 4 = the ciphertexts of mode 0, with
 * the rotations of every stage (2x2 window sums, horizontal and vertical
 * reductions) taken for all image shards together amount by amount, each key
 * read once per stage for up to 64 shards (channel shards and the fused
 * one-level reduction take mode 0).  Other modes: HEC_EINVAL.  Plans in modes
 * 2, 3 and 4 use the same mode for their stride-2 downsampling. */
hec_status he_avgpool_ex(hec_ctx *ctx, const hec_image *in, uint32_t window, int mode, hec_image **out);

/* Linear layer (Section 4.3, "Linear"): W is [O][C*H*W] over the input in
 * its logical [C][H][W] order (pool = 0), or [O][C] for the pool-linear layer
 * (pool = 1: global average pooling folded into the weights as W[o][f]/(H*W)
 * on every valid position of channel f).  Output o is the dot product of its
 * weights with the image: the shard products are summed and rescaled, the
 * slots summed by rotate-and-add (rotations N/2, ..., 2, 1, keys from
 * he_linear_steps), and the result masked onto slot o; the O masked results
 * are summed into *out (one ciphertext, two levels consumed, O <= N).  A
 * channel held in several blocks is read from its first block only. */
hec_status he_linear(hec_ctx *ctx, const hec_image *in, const double *W, uint32_t O, int pool, hec_ct **out);
hec_status he_linear_steps(hec_ctx *ctx, const hec_image *like, int32_t *steps, size_t cap, size_t *count);

/* Polynomial activation (Section 4.3 "GELU"; Appendix "Polynomial
 * Approximation"): p(x) = sum_k coeffs[k] T_k(y), y = (2x - a - b)/(b - a),
 * the Chebyshev expansion over [a, b] (degree ncoeffs - 1, 1..4095),
 * evaluated slotwise with the basis T_1 = y, T_{2k} = 2 T_k^2 - 1,
 * T_{2k+1} = 2 T_{k+1} T_k - T_1 up to the baby size m (smallest power of two
 * with m^2 > degree), giant powers T_{2m}, T_{4m}, ... and recursive division
 * by the largest giant power (T_j = 2 T_g T_{j-g} - T_{2g-j}).  Every product
 * is rescaled; the nominal scale of level l is S[l-1] = S[l]^2 / q_l from the
 * input's, constants multiply at S[l-1] q_l / S[l], level adjustments drop
 * limbs and multiply by 1.  Degree 59 consumes 7 levels.  Errors: HEC_EINVAL
 * (bad coefficients or interval, constant polynomial), HEC_ELEVEL (too few
 * levels), HEC_ENOKEY (no keys). */
hec_status he_cheb_eval(hec_ctx *ctx, const hec_ct *x, const double *coeffs, size_t ncoeffs, double a, double b,
                        hec_ct **out);
/* The same on every shard of an image (layout kept; slots outside the image
 * get p(0)). */
hec_status he_image_cheb_eval(hec_ctx *ctx, const hec_image *in, const double *coeffs, size_t ncoeffs, double a,
                              double b, hec_image **out);

/* Per-channel bias (the shift of an inference batch norm folded into the
 * preceding convolution, Section 4.3 "Batch Normalization"): bias[C] of the
 * image's logical channels, packed like the image (channel f's value on every
 * valid pixel of its blocks, zero elsewhere), encoded at each shard's level
 * and scale and added.  Shards must share level and scale. */
hec_status he_image_add_bias(hec_ctx *ctx, const hec_image *in, const double *bias, hec_image **out);

/* Basic block of the encrypted ResNets (Section 4.3; Section 4.1 and 4.2 for
 * its layers): conv k x k (w1 [C1][C][k][k], stride 1, padding k/2) with the
 * batch norm bn1 = [gamma[C1], shift[C1]] folded into weights and bias and
 * divided by `bound` (the map of [-bound, bound] onto [-1, 1]), the
 * activation as the Chebyshev series coeffs on [-1, 1] (for GELU: the
 * expansion of GELU(bound * y)), conv w2 [C2][C1][k][k] with bn2 folded (NULL:
 * no batch norm, no bias), 2x2 average pooling.  Folding: w'[o] = w[o] *
 * (gamma[o] / d), bias'[o] = shift[o] / d (d = bound, then 1).  mode as for
 * convolution plans (0..3); the pooling uses mode 2 or 3 when the block does,
 * else 0.  `like` fixes the input layout and level; he_block_steps lists the
 * rotation keys.  Levels: conv 1, activation (degree 59: 6), conv 1, pooling. */
hec_status he_block_create(hec_ctx *ctx, const hec_image *like, const double *w1, uint32_t C1, const double *bn1,
                           const double *w2, uint32_t C2, const double *bn2, uint32_t k, double bound,
                           const double *coeffs, size_t ncoeffs, int mode, hec_block **out);
hec_status he_block_steps(const hec_block *block, int32_t *steps, size_t cap, size_t *count);
hec_status he_block_run(hec_ctx *ctx, const hec_block *block, const hec_image *in, hec_image **out);
void he_block_free(hec_block *block);

/* ---- batches: many layer evaluations as one launch -------------------------
 * A batch lists (convolution plan, input image) items -- e.g. the images of
 * several requests, each at its own level and limb count, each through its 3x3
 * convolution and rescale (Section 4.1; the plan's mode applies).  Items keep
 * pointers to their plan and input, which must outlive the batch.
 * hec_batch_launch(HEC_BATCH_EAGER) runs the items one after another on the
 * context stream.  HEC_BATCH_GRAPH: the first launch runs the items once
 * eagerly on memory the batch keeps (so that the recording allocates
 * nothing), records them on a capture stream into one HIP graph and launches
 * it; later launches replay the graph on the context stream, re-reading the
 * inputs' current contents and rewriting the same outputs.  Ciphertexts are
 * the same bit for bit in both modes.  Items cannot be added after the
 * capture (HEC_EBUSY). */
typedef struct hec_batch hec_batch;
#define HEC_BATCH_EAGER 0
#define HEC_BATCH_GRAPH 1
hec_status hec_batch_begin(hec_ctx *ctx, hec_batch **out);
hec_status hec_batch_add(hec_batch *batch, const hec_conv_plan *plan, const hec_image *in, uint32_t *index);
hec_status hec_batch_launch(hec_batch *batch, int mode);
/* Borrowed output of item i from the last launch (eager outputs until the next
 * eager launch, graph outputs until hec_batch_free); NULL before a launch. */
const hec_image *hec_batch_output(const hec_batch *batch, uint32_t i);
uint32_t hec_batch_size(const hec_batch *batch);
/* Waits for the context stream, then frees the batch, its graph and memory. */
void hec_batch_free(hec_batch *batch);

/* ---- tuning: launch parameters and their autotuner -------------------------
 * Process-wide parameters that decide how work is cut into launches, never
 * its residues (every value gives the same ciphertexts bit for bit):
 *   ntt16_radix  16 | 2        2^16 transforms as two radix-16 register passes,
 *                              or as radix-2 stages over LDS tiles
 *   ntt_fp64     1 | 0         in the radix-16 form, the limbs of primes below
 *                              2^50 with exact double butterflies (every value
 *                              an integer below 2^52), or 64-bit integers
 *   ntt_row_vals 16 | 8        values per lane of the radix-16 form's forward
 *                              row pass (16: 256 lanes per 16-row tile, radix
 *                              16-16 rounds; 8: 512 lanes, radix 8-8-4)
 *   ntt_tile     2048 | 4096 | 8192   words per LDS tile of the radix-2 form
 *   ntt_group    0 | 64 | 256 | 1024  at most this many limbs per transform
 *                              launch (0: every limb of a batch in one launch)
 *   ks_rot_batch 4 | 8 | 16 | 32   rotations per key-switch launch of a hoisted set
 *   ks_overlap   0 | 1         a hoisted set's batches all on the context
 *                              stream, or alternating between it and a second
 *                              stream (forked and joined inside the call)
 *   ks_amounts   1 | 2 | 4 | 8 | 16   rotation amounts per key-stationary
 *                              launch (plan and pooling mode 4)
 * hec_tune_set rejects names and values outside these lists (HEC_EINVAL).
 * hec_tune_save / hec_tune_load persist them as "name value" lines. */
hec_status hec_tune_set(const char *name, int64_t value);
hec_status hec_tune_get(const char *name, int64_t *value);
/* "name=value ..." of every parameter (NUL-terminated; HEC_EINVAL if cap is too small). */
hec_status hec_tune_describe(char *buf, size_t cap);
hec_status hec_tune_save(const char *path);
hec_status hec_tune_load(const char *path);
/* Autotuner: times he_conv2d_plan_run(plan, in) (median of reps runs after an
 * untimed one) under every candidate of each parameter in turn, starting from
 * the current values; a candidate is kept only if the plan's output equals the
 * output under the starting values bit for bit and it is more than 2 % faster.
 * Leaves the chosen values set; report (nullable) receives the chosen values
 * and every timing.  Synchronizes. */
hec_status hec_autotune_conv(hec_ctx *ctx, const hec_conv_plan *plan, const hec_image *in, uint32_t reps,
                             char *report, size_t cap);

/* ---- serving: a request loop for encrypted inference ----------------------
 * Background, "Threat Model": the client encrypts its image and decrypts the
 * result, the server evaluates with the weights in the clear.  A server keeps
 * the context's evaluation and rotation keys and its models' plans resident
 * in HBM (generate every key the models need before hec_server_start) and
 * evaluates requests on `lanes` worker threads, each with its own HIP stream
 * and memory pool over the shared tables and keys, so that requests on
 * different lanes overlap on the device.  Admission is by device memory: a
 * model's footprint is the peak memory of one evaluation (measured by
 * hec_server_add_model, which also warms every lane); requests leave the queue
 * in arrival order while the footprints of the requests being evaluated stay
 * within mem_budget bytes; a request whose footprint alone exceeds the budget
 * is rejected (its poll returns HEC_ENOMEM).  Continuous batching: a lane
 * that frees up takes the oldest waiting request with the later waiting
 * requests of the same model (at most max_batch, as memory allows) and
 * evaluates them as one batch (plan mode 4: the rotations of all their shards
 * share each key read).  A request's ciphertexts do not depend on what it was
 * batched or overlapped with. */
typedef struct hec_server hec_server;
typedef struct {
    uint32_t lanes;       /* worker threads / HIP streams, 1..16 */
    uint32_t max_batch;   /* requests of one model evaluated together, >= 1 */
    size_t mem_budget;    /* device bytes for requests being evaluated */
} hec_server_params;
typedef struct {
    uint64_t completed, rejected, batches, batched_requests, max_concurrent;
    size_t peak_mem;                              /* largest sum of admitted footprints */
    double p50_ms, p99_ms, mean_ms, req_per_s;    /* latency submit -> done; completed per second */
} hec_server_stats_t;
hec_status hec_server_start(hec_ctx *ctx, const hec_server_params *params, hec_server **out);
/* A model: the convolution plan, then 2x2 average pooling in he_avgpool_ex
 * mode pool_mode (-1: none).  `like` is an input of the plan's layout and
 * level (evaluated once per lane).  Before the first submit (HEC_EBUSY after). */
hec_status hec_server_add_model(hec_server *server, const hec_conv_plan *plan, int pool_mode, const hec_image *like,
                                uint32_t *model);
size_t hec_server_model_footprint(const hec_server *server, uint32_t model);
/* Queue the evaluation of `in` (borrowed until its poll reports it done). */
hec_status hec_server_submit(hec_server *server, uint32_t model, const hec_image *in, uint64_t *request);
/* HEC_OK: done, *out receives the result (owned by the caller; free it with
 * hec_image_free before hec_server_stop, whose lanes own its memory) and
 * *latency_ms the time from submit to completion; HEC_EBUSY: not done yet
 * (wait = 0); any other status: the request failed (rejected: HEC_ENOMEM).
 * A request is reported once. */
hec_status hec_server_poll(hec_server *server, uint64_t request, int wait, hec_image **out, double *latency_ms);
hec_status hec_server_stats(hec_server *server, hec_server_stats_t *stats);
/* Evaluates what is queued, joins the workers and frees the server (and any
 * result not yet polled). */
hec_status hec_server_stop(hec_server *server);

void hec_ct_free(hec_ct *ct);
void hec_pt_free(hec_pt *pt);
void hec_image_free(hec_image *img);

/* Wait for all enqueued work of the context. */
hec_status hec_ctx_sync(hec_ctx *ctx);
/* Give the device memory the library keeps cached for reuse (its pools' free
 * blocks, on every context and serving lane of the device; not the memory of
 * live objects, keys, plans or captured batches) back to the device, after
 * the device's queued work.  Allocation does this by itself when HBM runs
 * short; the pools always leave 1 GiB of the device free for the runtime. */
hec_status hec_ctx_release_cached(hec_ctx *ctx);

/* ---- diagnostics ---------------------------------------------------------- */

/* Time every launch of the named kernel with HIP events on the context stream
 * until hec_prof_stop (one kernel at a time per process).  Names and units:
 * k_ntt16_fwd_cols, k_ntt16_inv_rows, k_ntt16_inv_cols (limbs transformed);
 * k_ntt16_fwd_rows (limbs moved to or from HBM: 2 per transformed limb, 3 in
 * the rescale form; in the ModDown form the product limb read, the rotated
 * limb written and what is added read); k_ks_inner, k_ks_inner_multi,
 * k_ks_mac (limbs moved: keys, plaintexts and outputs of every rotation,
 * shared digits and inputs once per launch); k_moddown_combine (rotation x
 * output limb); k_mac_terms (limb x term); k_bconv (polynomials); k_ew
 * (limbs).  Both calls synchronize the stream. */
hec_status hec_prof_start(hec_ctx *ctx, const char *kernel);
hec_status hec_prof_stop(hec_ctx *ctx, uint64_t *launches, uint64_t *units, double *total_ms);
/* Launches of the named kernel since the library was loaded (all contexts). */
uint64_t hec_prof_launches(const char *kernel);
/* Bandwidth probe: times a kernel that reads `nread` (1..8) and writes
 * `nwrite` (1..4) streams of `words` (256..2^32) 64-bit words, one word of
 * each stream per lane, non-temporal -- the access mix of a streaming kernel
 * without its arithmetic -- over `reps` (1..10000) launches after one
 * warm-up, on the context stream; *us_per_launch = the average duration in
 * microseconds (HIP events).  Allocates and frees its own (nread + nwrite) *
 * words * 8 bytes of device memory (HEC_ENOMEM if they do not fit);
 * synchronizes the stream; not for use under graph capture.  HEC_EINVAL for
 * counts out of range. */
hec_status hec_probe_stream(hec_ctx *ctx, int nread, int nwrite, uint64_t words, int reps, double *us_per_launch);
/* The thresholds of the discrete Gaussian sampler (Background, "Homomorphic
 * encryption": the error polynomials of keys and encryptions; sigma as in
 * hec_params): T[i] = floor(2^63 * sum_{|x| <= i} w(x) / sum_{|x| <= 19} w(x)),
 * w(x) = exp(-x^2 / (2 sigma^2)), i < 19; a draw takes the 63-bit value v and
 * returns the smallest i with v < T[i] (19 if none), signed by one more bit.
 * Host only (no device needed); cap >= 19; HEC_EINVAL for sigma outside
 * [2, 8], which hec_ctx_create rejects too. */
hec_status hec_gauss_table(double sigma, uint64_t *T, size_t cap);

#ifdef __cplusplus
}
#endif
#endif
