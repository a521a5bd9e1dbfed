// hec_internal.h -- host-side structures of the library (not part of the ABI).
#pragma once
#include <array>
#include <atomic>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/hecnn.h"
#include "hec_common.h"
#include "hec_host.h"

void hec_set_error(const char *fmt, ...);

#define HEC_TRY_HIP(expr)                                                                                          \
    do {                                                                                                           \
        hipError_t e_ = (expr);                                                                                    \
        if (e_ != hipSuccess) {                                                                                    \
            hec_set_error("HIP error %s at %s:%d", hipGetErrorString(e_), __FILE__, __LINE__);                      \
            return HEC_EDEVICE;                                                                                    \
        }                                                                                                          \
    } while (0)

#define HEC_FAIL(code, ...)                                                                                        \
    do {                                                                                                           \
        hec_set_error(__VA_ARGS__);                                                                                \
        return code;                                                                                               \
    } while (0)

#define HEC_CHECK(st)                                                                                              \
    do {                                                                                                           \
        hec_status s_ = (st);                                                                                      \
        if (s_ != HEC_OK) return s_;                                                                               \
    } while (0)

// Device memory pool: exact-size free lists; all users order their work on the
// context stream, so a block freed after enqueued work may be handed out again
// to later work on the same stream.  When the device is out of memory the
// cached blocks go back to it (after its queued work is done) and the
// allocation is tried once more.
// Thread-safe: a server's workers and its clients (freeing results) share pools.
// device memory the pools leave free for the runtime (queues, per-queue scratch)
#define HBM_RESERVE (1ull << 30)
// every trimmable pool of device dev gives its cached blocks back (after the
// device's queued work)
void trim_device_pools(int dev);
struct DevPool {
    std::unordered_multimap<size_t, void *> free_;
    std::unordered_map<void *, size_t> live_;
    size_t bytes_live = 0, bytes_cached = 0, peak_live = 0;
    std::mutex mu_;
    // When an allocation fails, every trimmable pool of the device gives its
    // cached blocks back (after the device's queued work) and the allocation
    // is tried once more.  A batch's pool is not trimmable: its cached blocks
    // are the temporaries of a captured graph that its replays still use.
    bool trimmable = true;
    std::atomic<int> dev{-1};  // device of the blocks (set at the first allocation)
    DevPool();
    ~DevPool();
    DevPool(const DevPool &) = delete;
    DevPool &operator=(const DevPool &) = delete;
    void *get(size_t bytes);
    bool put(void *p);  // false: not a block of this pool
    void trim();        // cached blocks back to the device (after the device's queued work)
    void release_cached();  // the same without waiting (the caller has synchronized)
    void release_all();
    size_t live()
    {
        std::lock_guard<std::mutex> lk(mu_);
        return bytes_live;
    }
};

struct Layout {
    uint32_t N = 0, C = 0, H = 0, W = 0, mp = 0;
    // image shards: per shard, block -> logical channel (-1 empty)
    std::vector<std::vector<int32_t>> maps;
    // channel shards (mp*mp > N): per shard, (channel, part); part v holds rows v*R .. v*R+R-1, R = N/mp
    bool channel = false;
    std::vector<std::pair<int32_t, int32_t>> cs;
    uint32_t B() const { return mp * mp; }
    uint32_t nb() const { return N / B(); }
    uint32_t R() const { return N / mp; }
    uint32_t spc() const { return B() / N; }
    size_t shards() const { return channel ? cs.size() : maps.size(); }
};

struct hec_ctx {
    hec_params prm{};
    int dev = 0;
    hipStream_t st = nullptr;
    // second stream (default priority) on which every other batch of a hoisted
    // rotation set runs, so that one batch's key switch (HBM-bound) overlaps
    // the previous batch's ModDown (transforms); forked from and joined back
    // into st by the two events; created at first use
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    uint32_t logn = 0, n = 0, N = 0, L = 0, k = 0, dnum = 0, alpha = 0, NLK = 0;
    std::vector<uint64_t> mod;
    DevPool pool;
    DevTables T{};
    // device tables
    PrimeC *d_pc = nullptr;
    u64 *d_tw = nullptr, *d_twsh = nullptr, *d_itw = nullptr, *d_itwsh = nullptr;
    double2 *d_twf = nullptr, *d_itwf = nullptr;
    u64 *d_z = nullptr, *d_zsh = nullptr;  // forward row-pass twists (n = 2^16)
    double *d_zf = nullptr;
    u32 *d_maps = nullptr;           // identity map (NLK) followed by QP maps of every level
    std::vector<size_t> qp_off;      // offset of level l's QP map in d_maps
    BconvDesc *d_modup = nullptr;    // [level][digit]
    BconvDesc *d_moddown = nullptr;  // [level]
    LevelC *d_lvl = nullptr;         // [level]
    u64 *d_pmodq = nullptr;          // [P]_{q_i}
    u64 *d_pmodq_m = nullptr;        // [P * 2^64]_{q_i}
    u64 *d_gauss = nullptr;
    u64 *d_crt_m = nullptr, *d_crt_inv = nullptr, *d_crt_invsh = nullptr;  // Garner tables (q primes)
    std::vector<BconvDesc> h_modup, h_moddown;
    double4 *d_enc_tw = nullptr;     // encoder twiddles cos/sin(pi e/n) as double-double, e < 2n
    u32 *d_enc_root = nullptr;       // FFT position of the root of each slot
    int *d_flag = nullptr;           // device status word (encoder overflow)
    // keys
    bool have_keys = false;
    uint64_t key_seed = 0;
    u64 *d_sN = nullptr, *d_sM = nullptr;  // secret, NTT form over all primes (plain / Montgomery)
    u64 *d_pk = nullptr;                   // [2][L+1][n] Montgomery
    std::map<uint32_t, u64 *> rotkeys;     // Galois element -> [dnum][2][NLK][n] Montgomery
    u64 *rlk = nullptr;                    // relinearization key (target s^2), same layout
    std::map<std::string, hec_pt *> mask_cache;
    std::map<uint32_t, u64 *> ones_qp;     // level -> the constant 1 over Q_l and P, Montgomery form
    uint64_t ks_count = 0;                 // key-switch inner products computed (one per rotation by g != 1)
    bool lane = false;                     // a serving lane: tables and keys belong to its parent
    std::mutex mu;

    const u32 *idmap() const { return d_maps; }
    const u32 *qpmap(uint32_t level) const { return d_maps + qp_off[level]; }
    size_t limb() const { return (size_t)n; }
    uint32_t galois(int64_t step) const;
    // where evaluation temporaries and results come from: the context's pool,
    // or the memory a captured graph keeps (hec_batch) while it records
    DevPool *active = &pool;
    u64 *alloc(size_t words) { return (u64 *)active->get(words * 8); }
    void release(void *p)
    {
        if (p && !active->put(p) && active != &pool) pool.put(p);
    }
};

// Routes the context's allocations to `p` for the scope (caches that outlive
// any batch are filled from the context's own pool).
struct PoolScope {
    hec_ctx *c;
    DevPool *prev;
    PoolScope(hec_ctx *c_, DevPool *p) : c(c_), prev(c_->active) { c->active = p; }
    ~PoolScope() { c->active = prev; }
};

struct hec_ct {
    hec_ctx *ctx = nullptr;
    uint32_t level = 0;
    double scale = 1.0;
    u64 *d = nullptr;  // [2][level+1][n], NTT form
};

struct hec_pt {
    hec_ctx *ctx = nullptr;
    uint32_t level = 0;
    double scale = 1.0;
    u64 *d = nullptr;  // [level+1 (+k)][n], NTT form, Montgomery; q_0..q_level then (optionally) p_0..p_{k-1}
    bool has_p = false;
    bool borrowed = false;  // d points into memory owned elsewhere (not released with the plaintext)
};

struct hec_image {
    hec_ctx *ctx = nullptr;
    Layout lay;
    std::vector<hec_ct *> shards;
};

// ---- internal API (hec_ctx.hip) -------------------------------------------
hec_ct *ct_new(hec_ctx *c, uint32_t level, double scale);
// a copy made on (allocated from and ordered on) context c
hec_ct *ct_clone(hec_ctx *c, const hec_ct *a);
// hoisted rotations of ct; D: ct's ModUp digits if the caller has them (from
// ct_modup of the same ciphertext, kept by the caller), else null: computed here
hec_status ct_rotate_hoisted(hec_ctx *c, const hec_ct *ct, const int32_t *steps, size_t n, hec_ct **outs,
                             const u64 *D = nullptr);
hec_status ct_rescale(hec_ctx *c, hec_ct *ct);
// every ciphertext (all at one level) rotated by `step`: one batched ModUp, key
// switch and ModDown; the same ciphertexts as one rotation at a time
hec_status ct_rotate_many(hec_ctx *c, const std::vector<const hec_ct *> &cts, int32_t step, std::vector<hec_ct *> &outs);
// key-stationary hoisted rotations of several ciphertexts at one level (ct_rotate_multi in hec_ctx.hip):
// want[a] bit u = input u needs amounts[a] (nonzero); the sink receives each batch of amounts' rotations,
// rots[(a - a0) * S + u] (null where not wanted), borrowed until it returns
typedef std::function<hec_status(size_t a0, size_t na, const std::vector<hec_ct *> &rots)> RotSink;
hec_status ct_rotate_multi(hec_ctx *c, const std::vector<const hec_ct *> &ins, const std::vector<int32_t> &amounts,
                           const std::vector<uint64_t> &want, size_t batch, const RotSink &sink);
// npolys polynomials [npolys][l+1][n] at level l divided by q_l (*d replaced by [npolys][l][n])
hec_status rescale_polys(hec_ctx *c, u64 **d, uint32_t l, int npolys);
// the per-limb residues of the integer r (and Shoup companions) for limbs 0..nlimbs-1
void scalar_arg(const hec_ctx *c, int64_t r, uint32_t nlimbs, ScalarArg &sa);
hec_status ct_add_inplace(hec_ctx *c, hec_ct *acc, const hec_ct *b);
// acc (+)= ct * pt ; first == true writes instead of accumulating
hec_status ct_mac_pt(hec_ctx *c, hec_ct *acc, const hec_ct *ct, const hec_pt *pt, bool first);
// encode many slot vectors (in parallel on the host) and upload; with_p also
// reduces the integer coefficients into the special primes (for products
// accumulated before ModDown)
hec_status pt_encode_many(hec_ctx *c, const std::vector<const double *> &z, size_t nz, uint32_t level, double scale,
                          std::vector<hec_pt *> &out, bool with_p = false);
// ModUp of c1 for hoisted key switching: *D = [beta][level+1+k][n] (NTT form), pool memory
hec_status ct_modup(hec_ctx *c, const hec_ct *ct, u64 **D);
// the same for several ciphertexts at one level in one set of launches: *Dall = [cnt][beta][level+1+k][n]
hec_status ct_modup_many(hec_ctx *c, const std::vector<const hec_ct *> &cts, u64 **Dall);
// out = ModDown(E), E = [2][level+1+k][n] over Q_l and P (NTT form); E's P limbs are overwritten
hec_status ct_moddown(hec_ctx *c, uint32_t level, u64 *E, hec_ct *out);
// outs[i] = ModDown(Eall + i * 2 (level+1+k) n) for several outputs (allocated at `level`) in one set of
// launches; with adds, (*adds)[i][p] ([level+1][n]) is added to polynomial p of output i in the same pass
hec_status ct_moddown_many(hec_ctx *c, uint32_t level, u64 *Eall, const std::vector<hec_ct *> &outs,
                           const std::vector<std::array<const u64 *, 2>> *adds = nullptr);
// the plaintext 1 over Q_l and P ([level+1+k][n], Montgomery form), cached per level
const u64 *ones_qp(hec_ctx *c, uint32_t level);
// the relinearization key (target s^2), generated from the key seed on first use
hec_status relin_key(hec_ctx *c, const u64 **key);
// ciphertext product with relinearization (not rescaled), scale a.scale * b.scale
hec_status ct_mul(hec_ctx *c, const hec_ct *a, const hec_ct *b, hec_ct **out);
// the constant polynomial round_half_away(value * scale) (exact product), |r| < 2^62
hec_status const_coeff(double value, double scale, int64_t *r);
// a * value (value encoded at pscale; result scale a.scale * pscale)
hec_status ct_mul_const(hec_ctx *c, const hec_ct *a, double value, double pscale, hec_ct **out);
// a + value (value encoded at `scale`)
hec_status ct_add_const(hec_ctx *c, const hec_ct *a, double value, double scale, hec_ct **out);
hec_status ct_sub(hec_ctx *c, const hec_ct *a, const hec_ct *b, hec_ct **out);
// a's first level+1 limbs (a dropped to `level`) * value at pscale
hec_status ct_mul_const_at(hec_ctx *c, const hec_ct *a, uint32_t level, double value, double pscale, hec_ct **out);
hec_status ct_drop(hec_ctx *c, const hec_ct *a, uint32_t level, hec_ct **out);
void pt_free(hec_pt *p);
void ct_free(hec_ct *p);
bool have_rotkey(hec_ctx *c, int32_t step);

// ct + pt (pt at the ciphertext's level and scale, without special-prime limbs)
hec_status ct_add_pt(hec_ctx *c, const hec_ct *a, const hec_pt *pt, hec_ct **out);

// serving lanes (hec_ctx.hip): contexts that share a parent's tables and keys
hec_status ctx_lane_create(hec_ctx *parent, hec_ctx **out);
void ctx_lane_destroy(hec_ctx *lane);

// ---- polynomial evaluation (hec_poly.cpp) ----------------------------------
// level and scale of the Chebyshev evaluation of a (level, scale) input, from a
// run over levels and scales only (also checks the constants and the level budget)
hec_status cheb_levels(hec_ctx *c, uint32_t level, double scale, const double *coeffs, size_t n, double a, double b,
                       uint32_t *out_level, double *out_scale);
// the evaluation of every ciphertext of `in` (new handles in out)
hec_status cheb_image(hec_ctx *c, const std::vector<hec_ct *> &in, const double *coeffs, size_t n, double a, double b,
                      std::vector<hec_ct *> &out);

// ---- layers (hec_layers.cpp) ---------------------------------------------
Layout natural_layout(uint32_t N, uint32_t C, uint32_t H, uint32_t W, uint32_t mp = 0);
// rotation steps of 2x2 pooling (select: the downsampling of a strided convolution) at `level`
void pool_steps(const Layout &L, bool select, uint32_t level, std::set<int32_t> &steps);
// convolution plan for an image of layout `lay` at `level` (what he_conv2d_plan_create builds from an image)
// basis > 0: weight plaintexts in basis-mask form with the masks encoded at 2^basis
hec_status conv_plan_create(hec_ctx *c, const Layout &lay, uint32_t level, const double *w, uint32_t Co, uint32_t kh,
                            uint32_t kw, uint32_t stride, uint32_t pad, hec_conv_plan **out, bool q_only = false,
                            uint32_t basis = 0);
// output layout of a plan (before the downsampling of a strided one)
const Layout &conv_plan_out(const hec_conv_plan *p);
// several images of a plan's layout and level, and the 2x2 pooling of several images of one layout,
// in one evaluation (key-stationary over all their shards in mode 4; image by image otherwise)
hec_status conv_plan_run_multi(hec_ctx *c, const hec_conv_plan *p, const std::vector<const hec_image *> &ins,
                               std::vector<hec_image *> &outs);
hec_status avgpool_multi(hec_ctx *c, const std::vector<const hec_image *> &ins, int mode,
                         std::vector<hec_image *> &outs);
// in + the per-channel bias (new handles in out)
hec_status image_add_bias(hec_ctx *c, const std::vector<hec_ct *> &in, const Layout &L, const double *bias,
                          std::vector<hec_ct *> &out);
