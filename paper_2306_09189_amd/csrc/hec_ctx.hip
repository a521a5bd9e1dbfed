// hec_ctx.hip -- context, keys and the RNS-CKKS ciphertext operations behind
// the C ABI (include/hecnn.h).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <thread>

#include "hec_internal.h"

using namespace hec;

// purposes of the random streams
enum { P_SECRET = 1, P_PK_A = 2, P_PK_E = 3, P_SWK_A = 4, P_SWK_E = 5, P_ENC_V = 6, P_ENC_E0 = 7, P_ENC_E1 = 8 };

static thread_local std::string g_err;
void hec_set_error(const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}
extern "C" const char *hec_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// pool
// ---------------------------------------------------------------------------
namespace {
// every pool of the process, so that a failed allocation can release the
// cached blocks of all pools of its device (never destroyed: pools may
// outlive the library's static objects at exit)
struct PoolRegistry {
    std::mutex mu;
    std::set<DevPool *> pools;
};
PoolRegistry &registry()
{
    static PoolRegistry *r = new PoolRegistry();
    return *r;
}
}  // namespace
void trim_device_pools(int dev)
{
    PoolRegistry &r = registry();
    std::lock_guard<std::mutex> lk(r.mu);
    (void)hipDeviceSynchronize();
    for (DevPool *p : r.pools)
        if (p->trimmable && p->dev.load() == dev) p->release_cached();
}

DevPool::DevPool()
{
    PoolRegistry &r = registry();
    std::lock_guard<std::mutex> lk(r.mu);
    r.pools.insert(this);
}
DevPool::~DevPool()
{
    PoolRegistry &r = registry();
    std::lock_guard<std::mutex> lk(r.mu);
    r.pools.erase(this);
}
void *DevPool::get(size_t bytes)
{
    if (!bytes) bytes = 8;
    void *p = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = free_.find(bytes);
        if (it != free_.end()) {
            p = it->second;
            free_.erase(it);
            bytes_cached -= bytes;
            live_[p] = bytes;
            bytes_live += bytes;
            peak_live = std::max(peak_live, bytes_live);
            return p;
        }
    }
    int d = 0;
    (void)hipGetDevice(&d);
    // The pools leave HBM_RESERVE of the device free for the runtime itself
    // (queues, and the scratch memory it allocates per queue at the first
    // launch of a kernel that needs it): when a block would cut into it, the
    // cached blocks of every pool of the device go back first, and if the
    // block still does not fit the allocation fails here with a null result
    // rather than leaving the runtime short later.
    auto fits = [&]() {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            return true;  // no figure: leave it to hipMalloc
        }
        return fr >= bytes + HBM_RESERVE;
    };
    bool ok = fits() && hipMalloc(&p, bytes) == hipSuccess;
    if (!ok) {
        // the failed call's error is cleared so that a later check of the launch status does not report it
        (void)hipGetLastError();
        trim_device_pools(d);
        if (!fits() || hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    std::lock_guard<std::mutex> lk(mu_);
    if (dev.load() < 0) dev.store(d);
    live_[p] = bytes;
    bytes_live += bytes;
    peak_live = std::max(peak_live, bytes_live);
    return p;
}
bool DevPool::put(void *p)
{
    std::lock_guard<std::mutex> lk(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) return false;
    free_.emplace(it->second, p);
    bytes_live -= it->second;
    bytes_cached += it->second;
    live_.erase(it);
    return true;
}
void DevPool::release_cached()
{
    std::lock_guard<std::mutex> lk(mu_);
    for (auto &kv : free_) hipFree(kv.second);
    free_.clear();
    bytes_cached = 0;
}
void DevPool::trim()
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (free_.empty()) return;
    }
    (void)hipDeviceSynchronize();
    release_cached();
}
void DevPool::release_all()
{
    std::lock_guard<std::mutex> lk(mu_);
    for (auto &kv : free_) hipFree(kv.second);
    for (auto &kv : live_) hipFree(kv.first);
    free_.clear();
    live_.clear();
    bytes_live = bytes_cached = 0;
}

// ---------------------------------------------------------------------------
// scratch of the allocation-free rotation (ckks_rotate_noalloc)
// ---------------------------------------------------------------------------
// One array per device: every GPU that loads the library holds its own copy
// until the process ends.  Host code never uses the array's name as an
// address: its device address is resolved once per device (with that device
// current) when a context is created there and kept in g_scratch_ptr.
#define HEC_MAX_DEVICES 64
static __device__ __align__(256) u64 scratch[HEC_NOALLOC_SCRATCH_BYTES / 8];
static u64 *g_scratch_ptr[HEC_MAX_DEVICES];
static std::mutex g_scratch_mu;

static hec_status scratch_init(int dev)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0 || dev >= HEC_MAX_DEVICES) HEC_FAIL(HEC_EDEVICE, "device %d beyond %d", dev, HEC_MAX_DEVICES);
    if (g_scratch_ptr[dev]) return HEC_OK;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        HEC_FAIL(HEC_EDEVICE, "scratch of the allocation-free rotation: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (u64 *)ptr;
    return HEC_OK;
}

uint32_t hec_ctx::galois(int64_t step) const
{
    int64_t r = step % (int64_t)N;
    if (r < 0) r += N;
    return (uint32_t)powmod(5, (uint64_t)r, 2ull * n);
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
static hec_status upload(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    HEC_TRY_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    return HEC_OK;
}

static uint32_t brv(uint32_t x, uint32_t bits)
{
    uint32_t r = 0;
    for (uint32_t i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

static hec_status build_tables(hec_ctx *c)
{
    const uint32_t n = c->n, NLK = c->NLK, L = c->L, k = c->k;
    const uint64_t r64_q = 0;
    (void)r64_q;
    // primes
    std::vector<PrimeC> pc(NLK);
    std::vector<u64> tw((size_t)NLK * n), twsh((size_t)NLK * n), itw((size_t)NLK * n), itwsh((size_t)NLK * n);
    std::vector<double2> twf((size_t)NLK * n), itwf((size_t)NLK * n);
    for (uint32_t i = 0; i < NLK; i++) {
        u64 q = c->mod[i];
        // -q^-1 mod 2^64 by Newton iteration
        u64 inv = 1;
        for (int it = 0; it < 7; it++) inv *= 2 - q * inv;
        pc[i].q = q;
        pc[i].qinv_neg = (u64)(0 - inv);
        u64 r1 = (u64)(((u128)1 << 64) % q);
        pc[i].r2 = mulmod(r1, r1, q);
        pc[i].ninv = invmod(n % q, q);
        pc[i].ninv_sh = shoup_of(pc[i].ninv, q);
        pc[i].fp = q < (1ull << 50) ? 1u : 0u;
        pc[i].qd = (double)q;
        pc[i].ninv_q = (double)pc[i].ninv / (double)q;
        pc[i].qinv_d = 1.0 / (double)q;
        u64 psi = find_root_2n(q, n), ipsi = invmod(psi, q);
        std::vector<u64> pw(n), ipw(n);
        pw[0] = ipw[0] = 1;
        for (uint32_t t = 1; t < n; t++) {
            pw[t] = mulmod(pw[t - 1], psi, q);
            ipw[t] = mulmod(ipw[t - 1], ipsi, q);
        }
        for (uint32_t t = 0; t < n; t++) {
            u64 w = pw[brv(t, c->logn)], iw = ipw[brv(t, c->logn)];
            tw[(size_t)i * n + t] = w;
            twsh[(size_t)i * n + t] = shoup_of(w, q);
            itw[(size_t)i * n + t] = iw;
            itwsh[(size_t)i * n + t] = shoup_of(iw, q);
            // w and w / q (each rounded to nearest) for the double butterflies
            twf[(size_t)i * n + t] = make_double2((double)w, (double)w / (double)q);
            itwf[(size_t)i * n + t] = make_double2((double)iw, (double)iw / (double)q);
        }
    }
    c->d_pc = (PrimeC *)c->pool.get(sizeof(PrimeC) * NLK);
    c->d_tw = c->alloc((size_t)NLK * n);
    c->d_twsh = c->alloc((size_t)NLK * n);
    c->d_itw = c->alloc((size_t)NLK * n);
    c->d_itwsh = c->alloc((size_t)NLK * n);
    c->d_twf = (double2 *)c->alloc((size_t)NLK * n * 2);
    c->d_itwf = (double2 *)c->alloc((size_t)NLK * n * 2);
    if (!c->d_pc || !c->d_tw || !c->d_twsh || !c->d_itw || !c->d_itwsh || !c->d_twf || !c->d_itwf)
        HEC_FAIL(HEC_ENOMEM, "table allocation");
    HEC_CHECK(upload(c->d_twf, twf.data(), twf.size() * sizeof(double2), c->st));
    HEC_CHECK(upload(c->d_itwf, itwf.data(), itwf.size() * sizeof(double2), c->st));
    HEC_CHECK(upload(c->d_pc, pc.data(), sizeof(PrimeC) * NLK, c->st));
    HEC_CHECK(upload(c->d_tw, tw.data(), tw.size() * 8, c->st));
    HEC_CHECK(upload(c->d_twsh, twsh.data(), twsh.size() * 8, c->st));
    HEC_CHECK(upload(c->d_itw, itw.data(), itw.size() * 8, c->st));
    HEC_CHECK(upload(c->d_itwsh, itwsh.data(), itwsh.size() * 8, c->st));
    if (c->logn == 16) {
        // Forward row-pass twists of the 2^16 transforms.  In the 256 x 256
        // view the twiddle of row-pass stage 8 + s, row r, butterfly group
        // t < 2^s is psi^brv16(2^(8+s) + r 2^s + t) = R_r^(2^(7-s)) psi^brv16(t)
        // with R_r = psi^(1 + 2 brv8(r)) (the three parts occupy disjoint
        // bits).  The factor R_r^(2^(7-s)) is met by the input at column c
        // exactly when bit 7-s of c is set, so over the whole pass it multiplies
        // that input by R_r^c: the pass is the element-wise product by R_r^c
        // followed by butterflies with the 128 row-independent twiddles
        // psi^brv16(t).  Same residues, one twist per element in place of the
        // row's own 255 twiddles.
        std::vector<u64> z((size_t)NLK * n), zsh((size_t)NLK * n);
        std::vector<double> zf((size_t)NLK * n);
        for (uint32_t i = 0; i < NLK; i++) {
            const u64 q = c->mod[i];
            const u64 psi = find_root_2n(q, n);
            std::vector<u64> pw(n);
            pw[0] = 1;
            for (uint32_t t = 1; t < n; t++) pw[t] = mulmod(pw[t - 1], psi, q);
            for (uint32_t r = 0; r < 256; r++)
                for (uint32_t col = 0; col < 256; col++) {
                    const uint64_t e = ((uint64_t)col * (1 + 2 * brv(r, 8))) % (2ull * n);  // psi^n = -1
                    const u64 w = e < n ? pw[e] : q - pw[e - n];
                    const size_t at = (size_t)i * n + r * 256 + col;
                    z[at] = w;
                    zsh[at] = shoup_of(w, q);
                    zf[at] = (double)w;
                }
        }
        c->d_z = c->alloc((size_t)NLK * n);
        c->d_zsh = c->alloc((size_t)NLK * n);
        c->d_zf = (double *)c->alloc((size_t)NLK * n);
        if (!c->d_z || !c->d_zsh || !c->d_zf) HEC_FAIL(HEC_ENOMEM, "table allocation");
        HEC_CHECK(upload(c->d_z, z.data(), z.size() * 8, c->st));
        HEC_CHECK(upload(c->d_zsh, zsh.data(), zsh.size() * 8, c->st));
        HEC_CHECK(upload(c->d_zf, zf.data(), zf.size() * 8, c->st));
        // the host vectors go out of scope below: the copies must have finished
        HEC_TRY_HIP(hipStreamSynchronize(c->st));
    }

    // limb -> prime maps: identity, then QP_l = q_0..q_l, p_0..p_{k-1} per level
    std::vector<u32> maps;
    for (uint32_t i = 0; i < NLK; i++) maps.push_back(i);
    c->qp_off.resize(L + 1);
    for (uint32_t l = 0; l <= L; l++) {
        c->qp_off[l] = maps.size();
        for (uint32_t i = 0; i <= l; i++) maps.push_back(i);
        for (uint32_t t = 0; t < k; t++) maps.push_back(L + 1 + t);
    }
    c->d_maps = (u32 *)c->pool.get(maps.size() * 4);
    HEC_CHECK(upload(c->d_maps, maps.data(), maps.size() * 4, c->st));

    // ModUp descriptors [level][digit] and ModDown descriptors [level]
    c->h_modup.assign((size_t)(L + 1) * c->dnum, BconvDesc{});
    c->h_moddown.assign(L + 1, BconvDesc{});
    std::vector<LevelC> lv(L + 1);
    for (uint32_t l = 0; l <= L; l++) {
        const uint32_t nq = l + 1, nqp = nq + k;
        std::vector<uint32_t> qp(nqp);
        for (uint32_t o = 0; o < nqp; o++) qp[o] = o < nq ? o : L + 1 + (o - nq);
        const uint32_t beta = (nq + c->alpha - 1) / c->alpha;
        for (uint32_t j = 0; j < beta; j++) {
            BconvDesc &d = c->h_modup[(size_t)l * c->dnum + j];
            uint32_t lo = j * c->alpha, hi = std::min((j + 1) * c->alpha, nq);
            d.nin = hi - lo;
            for (uint32_t a = 0; a < d.nin; a++) {
                uint32_t i = lo + a;
                u64 qi = c->mod[i], hat = 1;
                for (uint32_t b = lo; b < hi; b++)
                    if (b != i) hat = mulmod(hat, c->mod[b] % qi, qi);
                d.in_pos[a] = i;
                d.in_prime[a] = i;
                d.inv_hat[a] = invmod(hat, qi);
                d.inv_hat_sh[a] = shoup_of(d.inv_hat[a], qi);
            }
            d.nout = 0;
            for (uint32_t o = 0; o < nqp; o++) {
                if (o >= lo && o < hi) continue;
                d.out_pos[d.nout] = o;
                d.out_prime[d.nout] = qp[o];
                d.nout++;
            }
            for (uint32_t a = 0; a < d.nin; a++) {
                uint32_t i = lo + a;
                for (uint32_t b = 0; b < d.nout; b++) {
                    u64 t = c->mod[d.out_prime[b]], hat = 1;
                    for (uint32_t i2 = lo; i2 < hi; i2++)
                        if (i2 != i) hat = mulmod(hat, c->mod[i2] % t, t);
                    u64 r1 = (u64)(((u128)1 << 64) % t);
                    d.hat_m[a * d.nout + b] = mulmod(hat, r1, t);
                }
            }
        }
        // ModDown: inputs are the k P-limbs (positions nq..nq+k-1 of a QP_l buffer), outputs q_0..q_l
        BconvDesc &d = c->h_moddown[l];
        d.nin = k;
        for (uint32_t t = 0; t < k; t++) {
            u64 pt = c->mod[L + 1 + t], hat = 1;
            for (uint32_t t2 = 0; t2 < k; t2++)
                if (t2 != t) hat = mulmod(hat, c->mod[L + 1 + t2] % pt, pt);
            d.in_pos[t] = nq + t;
            d.in_prime[t] = L + 1 + t;
            d.inv_hat[t] = invmod(hat, pt);
            d.inv_hat_sh[t] = shoup_of(d.inv_hat[t], pt);
        }
        d.nout = nq;
        for (uint32_t i = 0; i < nq; i++) {
            d.out_pos[i] = i;
            d.out_prime[i] = i;
        }
        for (uint32_t t = 0; t < k; t++)
            for (uint32_t i = 0; i < nq; i++) {
                u64 qi = c->mod[i], hat = 1;
                for (uint32_t t2 = 0; t2 < k; t2++)
                    if (t2 != t) hat = mulmod(hat, c->mod[L + 1 + t2] % qi, qi);
                u64 r1 = (u64)(((u128)1 << 64) % qi);
                d.hat_m[t * nq + i] = mulmod(hat, r1, qi);
            }
        // rescale and ModDown scalars
        for (uint32_t i = 0; i < nq; i++) {
            u64 qi = c->mod[i];
            if (i < l) {
                lv[l].qlinv[i] = invmod(c->mod[l] % qi, qi);
                lv[l].qlinv_sh[i] = shoup_of(lv[l].qlinv[i], qi);
            }
            u64 P = 1;
            for (uint32_t t = 0; t < k; t++) P = mulmod(P, c->mod[L + 1 + t] % qi, qi);
            lv[l].pinv[i] = invmod(P, qi);
            lv[l].pinv_sh[i] = shoup_of(lv[l].pinv[i], qi);
        }
    }
    c->d_modup = (BconvDesc *)c->pool.get(sizeof(BconvDesc) * c->h_modup.size());
    c->d_moddown = (BconvDesc *)c->pool.get(sizeof(BconvDesc) * c->h_moddown.size());
    c->d_lvl = (LevelC *)c->pool.get(sizeof(LevelC) * lv.size());
    HEC_CHECK(upload(c->d_modup, c->h_modup.data(), sizeof(BconvDesc) * c->h_modup.size(), c->st));
    HEC_CHECK(upload(c->d_moddown, c->h_moddown.data(), sizeof(BconvDesc) * c->h_moddown.size(), c->st));
    HEC_CHECK(upload(c->d_lvl, lv.data(), sizeof(LevelC) * lv.size(), c->st));

    std::vector<u64> pm(NLK, 0);
    for (uint32_t i = 0; i <= L; i++) {
        u64 P = 1;
        for (uint32_t t = 0; t < k; t++) P = mulmod(P, c->mod[L + 1 + t] % c->mod[i], c->mod[i]);
        pm[i] = P;
    }
    c->d_pmodq = c->alloc(NLK);
    HEC_CHECK(upload(c->d_pmodq, pm.data(), NLK * 8, c->st));
    // P * 2^64 mod q_i (Montgomery form of P)
    std::vector<u64> pmm(NLK, 0);
    for (uint32_t i = 0; i <= L; i++) pmm[i] = (u64)(((u128)pm[i] << 64) % c->mod[i]);
    c->d_pmodq_m = c->alloc(NLK);
    HEC_CHECK(upload(c->d_pmodq_m, pmm.data(), NLK * 8, c->st));
    u64 gT[19];
    if (!gauss_table(c->prm.sigma, gT)) HEC_FAIL(HEC_EINVAL, "sigma must be in [2, 8]");
    c->d_gauss = c->alloc(19);
    HEC_CHECK(upload(c->d_gauss, gT, sizeof(gT), c->st));

    // Garner tables over q_0..q_L
    {
        std::vector<u64> Mm((size_t)HEC_MAX_LIMBS * HEC_MAX_LIMBS, 0), inv(HEC_MAX_LIMBS, 0), invsh(HEC_MAX_LIMBS, 0);
        for (uint32_t i = 0; i <= L; i++) {
            u64 qi = c->mod[i], r1 = (u64)(((u128)1 << 64) % qi), pr = 1;
            for (uint32_t j = 0; j < i; j++) {
                Mm[(size_t)i * HEC_MAX_LIMBS + j] = mulmod(pr, r1, qi);
                pr = mulmod(pr, c->mod[j] % qi, qi);
            }
            inv[i] = i ? invmod(pr, qi) : 1;
            invsh[i] = shoup_of(inv[i], qi);
        }
        c->d_crt_m = c->alloc(Mm.size());
        c->d_crt_inv = c->alloc(HEC_MAX_LIMBS);
        c->d_crt_invsh = c->alloc(HEC_MAX_LIMBS);
        if (!c->d_crt_m || !c->d_crt_inv || !c->d_crt_invsh) HEC_FAIL(HEC_ENOMEM, "table allocation");
        HEC_CHECK(upload(c->d_crt_m, Mm.data(), Mm.size() * 8, c->st));
        HEC_CHECK(upload(c->d_crt_inv, inv.data(), inv.size() * 8, c->st));
        HEC_CHECK(upload(c->d_crt_invsh, invsh.data(), invsh.size() * 8, c->st));
        {
            EncoderTables et(c->logn);
            c->d_enc_tw = (double4 *)c->pool.get(et.tw.size() * 8);
            c->d_enc_root = (u32 *)c->pool.get(et.root.size() * 4);
            c->d_flag = (int *)c->pool.get(256);
            if (!c->d_enc_tw || !c->d_enc_root || !c->d_flag) HEC_FAIL(HEC_ENOMEM, "table allocation");
            HEC_CHECK(upload(c->d_enc_tw, et.tw.data(), et.tw.size() * 8, c->st));
            HEC_CHECK(upload(c->d_enc_root, et.root.data(), et.root.size() * 4, c->st));
        }
        HEC_TRY_HIP(hipStreamSynchronize(c->st));
    }

    c->T.logn = c->logn;
    c->T.n = n;
    c->T.nprimes = NLK;
    c->T.pc = c->d_pc;
    c->T.tw = c->d_tw;
    c->T.tw_sh = c->d_twsh;
    c->T.itw = c->d_itw;
    c->T.itw_sh = c->d_itwsh;
    c->T.twf = c->d_twf;
    c->T.itwf = c->d_itwf;
    c->T.z = c->d_z;
    c->T.z_sh = c->d_zsh;
    c->T.zf = c->d_zf;
    c->T.fp_on = 1;
    HEC_TRY_HIP(hipStreamSynchronize(c->st));
    return HEC_OK;
}

extern "C" hec_status hec_ctx_create(const hec_params *p, int device, void *hip_stream, hec_ctx **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) HEC_FAIL(HEC_EINVAL, "params is NULL");
    if (p->log_n < 5 || p->log_n > 16) HEC_FAIL(HEC_EINVAL, "log_n must be in [5, 16]");
    if (p->L + 1 + p->k > HEC_MAX_LIMBS) HEC_FAIL(HEC_EINVAL, "too many primes");
    if (p->k < 1 || p->k > HEC_MAX_BCONV_IN) HEC_FAIL(HEC_EINVAL, "need 1..16 special primes");
    for (uint32_t b : {p->q0_bits, p->q_bits, p->p_bits})
        if (b < 20 || b > 60) HEC_FAIL(HEC_EINVAL, "prime sizes must be in [20, 60] bits");
    if (p->dnum < 1 || p->dnum > p->L + 1) HEC_FAIL(HEC_EINVAL, "dnum must be in [1, L+1]");
    uint32_t alpha = (p->L + 1 + p->dnum - 1) / p->dnum;
    if (alpha > HEC_MAX_BCONV_IN) HEC_FAIL(HEC_EINVAL, "digits larger than 16 primes are not supported");
    if (p->secret_dist != 0) HEC_FAIL(HEC_EINVAL, "only the uniform ternary secret is supported");
    if (!(p->sigma >= 2.0 && p->sigma <= 8.0)) HEC_FAIL(HEC_EINVAL, "sigma must be in [2, 8]");
    int ndev = 0;
    HEC_TRY_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) HEC_FAIL(HEC_EDEVICE, "no HIP device %d", device);
    HEC_TRY_HIP(hipSetDevice(device));
    HEC_CHECK(scratch_init(device));

    std::unique_ptr<hec_ctx> c(new hec_ctx());
    c->prm = *p;
    c->dev = device;
    c->st = (hipStream_t)hip_stream;
    c->logn = p->log_n;
    c->n = 1u << p->log_n;
    c->N = c->n / 2;
    c->L = p->L;
    c->k = p->k;
    c->alpha = alpha;
    c->dnum = (p->L + 1 + alpha - 1) / alpha;
    c->NLK = p->L + 1 + p->k;
    std::vector<uint64_t> taken;
    for (uint32_t i = 0; i < c->NLK; i++) {
        uint32_t b = i == 0 ? p->q0_bits : (i <= p->L ? p->q_bits : p->p_bits);
        uint64_t q = find_prime(b, c->n, taken);
        if (!q) HEC_FAIL(HEC_EINVAL, "no %u-bit prime = 1 mod 2n left", b);
        taken.push_back(q);
    }
    c->mod = taken;
    // the exact 128-bit accumulations need m * q_max < 2^64 for m terms of products
    // below q^2: alpha (ModUp), k (ModDown), dnum + 1 (key switch with the folded
    // c0 term) and HEC_KS_BATCH (fused plaintext products)
    const uint32_t mterms = std::max(std::max(alpha, c->k), std::max(c->dnum + 1, (uint32_t)HEC_KS_BATCH));
    for (uint64_t q : c->mod)
        if ((u128)q * mterms >= ((u128)1 << 64)) HEC_FAIL(HEC_EINVAL, "primes too large for digits");
    hec_status s = build_tables(c.get());
    if (s != HEC_OK) {
        c->pool.release_all();
        return s;
    }
    *out = c.release();
    return HEC_OK;
}

static void side_release(hec_ctx *c)
{
    if (c->side) {
        hipStreamSynchronize(c->side);
        hipStreamDestroy(c->side);
    }
    if (c->ev_fork) hipEventDestroy(c->ev_fork);
    if (c->ev_join) hipEventDestroy(c->ev_join);
    c->side = nullptr;
    c->ev_fork = c->ev_join = nullptr;
}
// the side stream and its events, created at first use
static hec_status side_stream(hec_ctx *c)
{
    if (c->side) return HEC_OK;
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&a, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (s) hipStreamDestroy(s);
        if (a) hipEventDestroy(a);
        HEC_FAIL(HEC_EDEVICE, "side stream: %s", hipGetErrorString(e));
    }
    c->side = s;
    c->ev_fork = a;
    c->ev_join = b;
    return HEC_OK;
}

extern "C" void hec_ctx_destroy(hec_ctx *c)
{
    if (!c) return;
    hipSetDevice(c->dev);
    hipStreamSynchronize(c->st);
    side_release(c);
    c->pool.release_all();
    delete c;
}

// A serving lane: everything read-only of `parent` shared (tables, keys), its
// own stream, memory pool, encoder status word and caches, so that one worker
// thread per lane evaluates concurrently with the others.
hec_status ctx_lane_create(hec_ctx *parent, hec_ctx **out)
{
    *out = nullptr;
    HEC_TRY_HIP(hipSetDevice(parent->dev));
    std::unique_ptr<hec_ctx> c(new hec_ctx());
    c->prm = parent->prm;
    c->dev = parent->dev;
    c->logn = parent->logn; c->n = parent->n; c->N = parent->N; c->L = parent->L; c->k = parent->k;
    c->dnum = parent->dnum; c->alpha = parent->alpha; c->NLK = parent->NLK;
    c->mod = parent->mod;
    c->T = parent->T;
    c->d_pc = parent->d_pc;
    c->d_tw = parent->d_tw; c->d_twsh = parent->d_twsh; c->d_itw = parent->d_itw; c->d_itwsh = parent->d_itwsh;
    c->d_twf = parent->d_twf; c->d_itwf = parent->d_itwf;
    c->d_z = parent->d_z; c->d_zsh = parent->d_zsh; c->d_zf = parent->d_zf;
    c->d_maps = parent->d_maps;
    c->qp_off = parent->qp_off;
    c->d_modup = parent->d_modup; c->d_moddown = parent->d_moddown; c->d_lvl = parent->d_lvl;
    c->d_pmodq = parent->d_pmodq; c->d_pmodq_m = parent->d_pmodq_m; c->d_gauss = parent->d_gauss;
    c->d_crt_m = parent->d_crt_m; c->d_crt_inv = parent->d_crt_inv; c->d_crt_invsh = parent->d_crt_invsh;
    c->h_modup = parent->h_modup; c->h_moddown = parent->h_moddown;
    c->d_enc_tw = parent->d_enc_tw; c->d_enc_root = parent->d_enc_root;
    c->have_keys = parent->have_keys; c->key_seed = parent->key_seed;
    c->d_sN = parent->d_sN; c->d_sM = parent->d_sM; c->d_pk = parent->d_pk;
    c->rotkeys = parent->rotkeys;
    c->rlk = parent->rlk;
    c->lane = true;
    HEC_TRY_HIP(hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking));
    c->d_flag = (int *)c->pool.get(256);
    if (!c->d_flag) {
        hipStreamDestroy(c->st);
        HEC_FAIL(HEC_ENOMEM, "lane status word");
    }
    *out = c.release();
    return HEC_OK;
}

void ctx_lane_destroy(hec_ctx *c)
{
    if (!c) return;
    hipSetDevice(c->dev);
    hipStreamSynchronize(c->st);
    side_release(c);
    hipStreamDestroy(c->st);
    c->pool.release_all();
    delete c;
}

extern "C" hec_status hec_ctx_sync(hec_ctx *c)
{
    if (!c) HEC_FAIL(HEC_EINVAL, "ctx is NULL");
    HEC_TRY_HIP(hipStreamSynchronize(c->st));
    return HEC_OK;
}

extern "C" hec_status hec_ctx_release_cached(hec_ctx *c)
{
    if (!c) HEC_FAIL(HEC_EINVAL, "ctx is NULL");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    trim_device_pools(c->dev);
    HEC_TRY_HIP(hipGetLastError());
    return HEC_OK;
}

extern "C" hec_status hec_ctx_primes(const hec_ctx *c, uint64_t *primes, size_t cap, size_t *count)
{
    if (!c) HEC_FAIL(HEC_EINVAL, "ctx is NULL");
    if (count) *count = c->mod.size();
    if (primes) {
        if (cap < c->mod.size()) HEC_FAIL(HEC_EINVAL, "capacity too small");
        memcpy(primes, c->mod.data(), c->mod.size() * 8);
    }
    return HEC_OK;
}

extern "C" uint32_t hec_ctx_slots(const hec_ctx *c) { return c ? c->N : 0; }

extern "C" hec_status hec_gauss_table(double sigma, uint64_t *T, size_t cap)
{
    if (!T || cap < 19) HEC_FAIL(HEC_EINVAL, "the table has 19 entries");
    u64 t[19];
    if (!gauss_table(sigma, t)) HEC_FAIL(HEC_EINVAL, "sigma must be in [2, 8]");
    memcpy(T, t, sizeof(t));
    return HEC_OK;
}

extern "C" uint64_t hec_ctx_keyswitch_count(const hec_ctx *c) { return c ? c->ks_count : 0; }

extern "C" size_t hec_ctx_key_bytes(const hec_ctx *c)
{
    return c ? (c->rotkeys.size() + (c->rlk ? 1 : 0)) * (size_t)c->dnum * 2 * c->NLK * c->n * 8 : 0;
}

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
hec_ct *ct_new(hec_ctx *c, uint32_t level, double scale)
{
    u64 *d = c->alloc((size_t)2 * (level + 1) * c->n);
    if (!d) return nullptr;
    hec_ct *ct = new hec_ct();
    ct->ctx = c;
    ct->level = level;
    ct->scale = scale;
    ct->d = d;
    return ct;
}
hec_ct *ct_clone(hec_ctx *c, const hec_ct *a)
{
    hec_ct *r = ct_new(c, a->level, a->scale);
    if (!r) return nullptr;
    hipMemcpyAsync(r->d, a->d, (size_t)2 * (a->level + 1) * c->n * 8, hipMemcpyDeviceToDevice, c->st);
    return r;
}
void ct_free(hec_ct *p)
{
    if (!p) return;
    p->ctx->release(p->d);
    delete p;
}
void pt_free(hec_pt *p)
{
    if (!p) return;
    if (!p->borrowed) p->ctx->release(p->d);
    delete p;
}
extern "C" void hec_ct_free(hec_ct *ct) { ct_free(ct); }
extern "C" void hec_pt_free(hec_pt *pt) { pt_free(pt); }

extern "C" hec_status ckks_ct_info(const hec_ct *ct, uint32_t *level, double *scale)
{
    if (!ct) HEC_FAIL(HEC_EINVAL, "ct is NULL");
    if (level) *level = ct->level;
    if (scale) *scale = ct->scale;
    return HEC_OK;
}

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------
// Key-switching key to s for Galois element g (target sigma_g(s)); with tgt
// (NTT form, all primes) the target is tgt instead and g = 0 (the
// relinearization key, target s^2): random streams (g << 8) | digit.
static hec_status gen_swk(hec_ctx *c, uint32_t g, const u64 *tgt = nullptr, u64 **out = nullptr)
{
    if (!tgt && c->rotkeys.count(g)) return HEC_OK;
    PoolScope ps(c, &c->pool);  // keys live as long as the context
    const size_t n = c->n, NLK = c->NLK;
    u64 *key = c->alloc((size_t)c->dnum * 2 * NLK * n);
    u64 *e = c->alloc(NLK * n);
    int64_t *es = (int64_t *)c->alloc(n);
    if (!key || !e || !es) HEC_FAIL(HEC_ENOMEM, "rotation key allocation");
    for (uint32_t j = 0; j < c->dnum; j++) {
        u64 *b = key + (size_t)j * 2 * NLK * n, *a = b + NLK * n;
        uint64_t idx = ((uint64_t)g << 8) | j;
        hec_sample_uniform(c->T, a, c->key_seed, P_SWK_A, idx, c->idmap(), NLK, c->st);
        hec_ntt_fwd(c->T, a, 0, 1, c->idmap(), NLK, c->st);
        hec_sample_small(c->T, es, c->key_seed, P_SWK_E, idx, 1, c->d_gauss, c->st);
        hec_reduce_i64(c->T, e, es, c->idmap(), NLK, c->st);
        hec_ntt_fwd(c->T, e, 0, 1, c->idmap(), NLK, c->st);
        uint32_t dlo = j * c->alpha, dhi = std::min((j + 1) * c->alpha, c->L + 1);
        hec_key_finish(c->T, b, a, e, c->d_sN, tgt, c->d_pmodq, g, dlo, dhi, NLK, c->idmap(), c->st);
    }
    c->release(e);
    c->release(es);
    HEC_TRY_HIP(hipGetLastError());
    if (out) *out = key;
    else c->rotkeys[g] = key;
    return HEC_OK;
}

// relinearization key (target s^2), generated on first use from the key seed
hec_status relin_key(hec_ctx *c, const u64 **key)
{
    if (!c->have_keys) HEC_FAIL(HEC_ENOKEY, "no keys");
    if (!c->rlk) {
        PoolScope ps(c, &c->pool);
        const size_t n = c->n, NLK = c->NLK;
        u64 *s2 = c->alloc(NLK * n);
        if (!s2) HEC_FAIL(HEC_ENOMEM, "key allocation");
        hec_ew(c->T, EW_MUL_MONT, s2, c->d_sN, c->d_sM, 0, 0, 0, 1, c->idmap(), (int)NLK, c->st);
        hec_status s = gen_swk(c, 0, s2, &c->rlk);
        c->release(s2);
        HEC_CHECK(s);
    }
    *key = c->rlk;
    return HEC_OK;
}

extern "C" hec_status ckks_keygen(hec_ctx *c, uint64_t seed, const int32_t *steps, size_t nsteps)
{
    if (!c) HEC_FAIL(HEC_EINVAL, "ctx is NULL");
    if (nsteps && !steps) HEC_FAIL(HEC_EINVAL, "steps is NULL");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    const size_t n = c->n, NLK = c->NLK, nq = c->L + 1;
    for (auto &kv : c->rotkeys) c->release(kv.second);
    c->rotkeys.clear();
    c->release(c->rlk);
    c->rlk = nullptr;
    for (auto &kv : c->mask_cache) pt_free(kv.second);
    c->mask_cache.clear();
    c->key_seed = seed;
    if (!c->d_sN) {
        c->d_sN = c->alloc(NLK * n);
        c->d_sM = c->alloc(NLK * n);
        c->d_pk = c->alloc(2 * nq * n);
    }
    int64_t *sm = (int64_t *)c->alloc(n);
    u64 *e = c->alloc(nq * n);
    if (!c->d_sN || !c->d_sM || !c->d_pk || !sm || !e) HEC_FAIL(HEC_ENOMEM, "key allocation");
    hec_sample_small(c->T, sm, seed, P_SECRET, 0, 0, c->d_gauss, c->st);
    hec_reduce_i64(c->T, c->d_sN, sm, c->idmap(), NLK, c->st);
    hec_ntt_fwd(c->T, c->d_sN, 0, 1, c->idmap(), NLK, c->st);
    hec_ew(c->T, EW_TO_MONT, c->d_sM, c->d_sN, nullptr, 0, 0, 0, 1, c->idmap(), NLK, c->st);
    // pk = (-a s + e, a)
    u64 *b = c->d_pk, *a = c->d_pk + nq * n;
    hec_sample_uniform(c->T, a, seed, P_PK_A, 0, c->idmap(), nq, c->st);
    hec_ntt_fwd(c->T, a, 0, 1, c->idmap(), nq, c->st);
    hec_sample_small(c->T, sm, seed, P_PK_E, 0, 1, c->d_gauss, c->st);
    hec_reduce_i64(c->T, e, sm, c->idmap(), nq, c->st);
    hec_ntt_fwd(c->T, e, 0, 1, c->idmap(), nq, c->st);
    hec_key_finish(c->T, b, a, e, c->d_sN, nullptr, nullptr, 1, 0, 0, nq, c->idmap(), c->st);
    c->release(sm);
    c->release(e);
    HEC_TRY_HIP(hipGetLastError());
    c->have_keys = true;
    return ckks_gen_rotation_keys(c, steps, nsteps);
}

extern "C" hec_status ckks_gen_rotation_keys(hec_ctx *c, const int32_t *steps, size_t nsteps)
{
    if (!c) HEC_FAIL(HEC_EINVAL, "ctx is NULL");
    if (!c->have_keys) HEC_FAIL(HEC_ENOKEY, "ckks_keygen has not been called");
    if (nsteps && !steps) HEC_FAIL(HEC_EINVAL, "steps is NULL");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    for (size_t i = 0; i < nsteps; i++) {
        uint32_t g = c->galois(steps[i]);
        if (g == 1) continue;
        HEC_CHECK(gen_swk(c, g));
    }
    return HEC_OK;
}

bool have_rotkey(hec_ctx *c, int32_t step)
{
    uint32_t g = c->galois(step);
    return g == 1 || c->rotkeys.count(g);
}

// ---------------------------------------------------------------------------
// encoding
// ---------------------------------------------------------------------------
// signed integer coefficients (device) -> plaintext limbs over q_0..q_level
// (and p_0..p_{k-1} when with_p), evaluation + Montgomery form
static hec_status make_pt(hec_ctx *c, const int64_t *dm, uint32_t level, double scale, bool with_p, hec_pt **out)
{
    const size_t n = c->n, nl = level + 1 + (with_p ? c->k : 0);
    const u32 *pmap = with_p ? c->qpmap(level) : c->idmap();
    u64 *d = c->alloc(nl * n);
    if (!d) HEC_FAIL(HEC_ENOMEM, "plaintext allocation");
    hec_reduce_i64(c->T, d, dm, pmap, (int)nl, c->st);
    hec_ntt_fwd(c->T, d, 0, 1, pmap, (int)nl, c->st);
    hec_ew(c->T, EW_TO_MONT, d, d, nullptr, 0, 0, 0, 1, pmap, (int)nl, c->st);
    hec_pt *p = new hec_pt();
    p->ctx = c;
    p->level = level;
    p->scale = scale;
    p->d = d;
    p->has_p = with_p;
    *out = p;
    return HEC_OK;
}

// encode `count` slot vectors held in device memory (stride zstride, nz values
// each) into signed coefficients dm[count][n] on the device; waits for the
// result of the overflow check
static hec_status encode_device(hec_ctx *c, const double *dz, size_t zstride, size_t nz, size_t count, double scale,
                                int64_t *dm)
{
    const size_t n = c->n;
    double4 *work = (double4 *)c->pool.get(count * n * sizeof(double4));
    if (!work) HEC_FAIL(HEC_ENOMEM, "encoder buffer");
    hec_encode(dz, zstride, (u32)nz, (u32)count, scale, c->d_enc_root, c->d_enc_tw, work, dm, c->d_flag, c->logn,
               c->st);
    int flag = 0;
    hipError_t e = hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    c->pool.put(work);
    if (e != hipSuccess) HEC_FAIL(HEC_EDEVICE, "encoder: %s", hipGetErrorString(e));
    if (flag) HEC_FAIL(HEC_EINVAL, "encoded coefficient exceeds 2^62 (scale too large for the values)");
    return HEC_OK;
}

hec_status pt_encode_many(hec_ctx *c, const std::vector<const double *> &z, size_t nz, uint32_t level, double scale,
                          std::vector<hec_pt *> &out, bool with_p)
{
    const size_t cnt = z.size(), n = c->n, N = c->N;
    out.assign(cnt, nullptr);
    // slot vectors staged through the device in chunks; encoding, reduction and
    // NTT all run there
    const size_t chunk = 64, cmax = std::min(cnt, chunk);
    std::vector<double> hz(cmax * N, 0.0);
    double *dz = (double *)c->pool.get(cmax * N * 8);
    int64_t *dm = (int64_t *)c->alloc(cmax * n);
    hec_status s = (dz && dm) ? HEC_OK : HEC_ENOMEM;
    if (s != HEC_OK) hec_set_error("encoder staging allocation");
    for (size_t i0 = 0; i0 < cnt && s == HEC_OK; i0 += chunk) {
        const size_t cc = std::min(chunk, cnt - i0);
        for (size_t i = 0; i < cc; i++) memcpy(&hz[i * N], z[i0 + i], nz * 8);
        if (hipMemcpyAsync(dz, hz.data(), cc * N * 8, hipMemcpyHostToDevice, c->st) != hipSuccess) {
            s = HEC_EDEVICE;
            hec_set_error("plaintext upload failed");
            break;
        }
        // encode_device waits for the stream, so hz may be refilled afterwards
        s = encode_device(c, dz, N, nz, cc, scale, dm);
        for (size_t i = 0; i < cc && s == HEC_OK; i++) s = make_pt(c, dm + i * n, level, scale, with_p, &out[i0 + i]);
    }
    // make_pt's kernels read dm: order the release after them on the stream
    c->pool.put(dz);
    c->release(dm);
    if (s != HEC_OK) {
        for (auto *p : out) pt_free(p);
        out.clear();
    }
    return s;
}

extern "C" hec_status ckks_encode_coeffs(hec_ctx *c, const double *z, size_t nz, double scale, int64_t *m)
{
    if (!c || !m || (nz && !z)) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (nz > c->N) HEC_FAIL(HEC_EINVAL, "more values than slots");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    const size_t n = c->n;
    double *dz = (double *)c->pool.get(c->N * 8);
    int64_t *dm = (int64_t *)c->alloc(n);
    if (!dz || !dm) {
        c->pool.put(dz);
        c->release(dm);
        HEC_FAIL(HEC_ENOMEM, "encoder staging allocation");
    }
    hec_status s = HEC_OK;
    if (nz && hipMemcpyAsync(dz, z, nz * 8, hipMemcpyHostToDevice, c->st) != hipSuccess) s = HEC_EDEVICE;
    if (s == HEC_OK) s = encode_device(c, dz, c->N, nz, 1, scale, dm);
    if (s == HEC_OK && (hipMemcpyAsync(m, dm, n * 8, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
                        hipStreamSynchronize(c->st) != hipSuccess))
        s = HEC_EDEVICE;
    c->pool.put(dz);
    c->release(dm);
    if (s == HEC_EDEVICE) hec_set_error("encoder transfer failed");
    return s;
}

extern "C" hec_status ckks_encode(hec_ctx *c, const double *z, size_t nz, uint32_t level, double scale, hec_pt **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || (nz && !z)) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (nz > c->N) HEC_FAIL(HEC_EINVAL, "more values than slots");
    if (level > c->L) HEC_FAIL(HEC_ELEVEL, "level above L");
    if (!(scale > 0)) HEC_FAIL(HEC_EINVAL, "scale must be positive");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    std::vector<hec_pt *> v;
    HEC_CHECK(pt_encode_many(c, {z}, nz, level, scale, v));
    *out = v[0];
    return HEC_OK;
}

extern "C" hec_status ckks_pt_import(hec_ctx *c, const uint64_t *coeff, uint32_t level, double scale, hec_pt **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !coeff) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (level > c->L) HEC_FAIL(HEC_ELEVEL, "level above L");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    const size_t n = c->n, nq = level + 1;
    for (size_t i = 0; i < nq; i++)
        for (size_t t = 0; t < n; t++)
            if (coeff[i * n + t] >= c->mod[i]) HEC_FAIL(HEC_EINVAL, "residue not reduced");
    u64 *d = c->alloc(nq * n);
    if (!d) HEC_FAIL(HEC_ENOMEM, "plaintext allocation");
    HEC_TRY_HIP(hipMemcpyAsync(d, coeff, nq * n * 8, hipMemcpyHostToDevice, c->st));
    hec_ntt_fwd(c->T, d, 0, 1, c->idmap(), nq, c->st);
    hec_ew(c->T, EW_TO_MONT, d, d, nullptr, 0, 0, 0, 1, c->idmap(), nq, c->st);
    HEC_TRY_HIP(hipStreamSynchronize(c->st));
    hec_pt *p = new hec_pt();
    p->ctx = c;
    p->level = level;
    p->scale = scale;
    p->d = d;
    *out = p;
    return HEC_OK;
}

extern "C" hec_status ckks_pt_export(hec_ctx *c, const hec_pt *pt, uint64_t *coeff, uint32_t *level, double *scale)
{
    if (!c || !pt || !coeff) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    const size_t n = c->n, nq = pt->level + 1;
    u64 *t = c->alloc(nq * n);
    if (!t) HEC_FAIL(HEC_ENOMEM, "export buffer");
    hec_ew(c->T, EW_FROM_MONT, t, pt->d, nullptr, 0, 0, 0, 1, c->idmap(), nq, c->st);
    hec_ntt_inv(c->T, t, 0, 1, c->idmap(), nq, c->st);
    HEC_TRY_HIP(hipMemcpyAsync(coeff, t, nq * n * 8, hipMemcpyDeviceToHost, c->st));
    HEC_TRY_HIP(hipStreamSynchronize(c->st));
    c->release(t);
    if (level) *level = pt->level;
    if (scale) *scale = pt->scale;
    return HEC_OK;
}

// ---------------------------------------------------------------------------
// encryption / decryption
// ---------------------------------------------------------------------------
extern "C" hec_status ckks_encrypt_idx(hec_ctx *c, const hec_pt *pt, uint64_t seed, uint64_t index, hec_ct **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !pt) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (!c->have_keys) HEC_FAIL(HEC_ENOKEY, "no public key (call ckks_keygen)");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    const size_t n = c->n, nq = pt->level + 1;
    hec_ct *ct = ct_new(c, pt->level, pt->scale);
    u64 *buf = c->alloc(4 * nq * n);
    int64_t *sm = (int64_t *)c->alloc(n);
    if (!ct || !buf || !sm) HEC_FAIL(HEC_ENOMEM, "encryption buffers");
    u64 *v = buf, *e0 = buf + nq * n, *e1 = buf + 2 * nq * n, *m = buf + 3 * nq * n;
    hec_sample_small(c->T, sm, seed, P_ENC_V, index, 0, c->d_gauss, c->st);
    hec_reduce_i64(c->T, v, sm, c->idmap(), nq, c->st);
    hec_sample_small(c->T, sm, seed, P_ENC_E0, index, 1, c->d_gauss, c->st);
    hec_reduce_i64(c->T, e0, sm, c->idmap(), nq, c->st);
    hec_sample_small(c->T, sm, seed, P_ENC_E1, index, 1, c->d_gauss, c->st);
    hec_reduce_i64(c->T, e1, sm, c->idmap(), nq, c->st);
    hec_ntt_fwd(c->T, buf, 0, 1, c->idmap(), nq, c->st);
    hec_ntt_fwd(c->T, e0, 0, 1, c->idmap(), nq, c->st);
    hec_ntt_fwd(c->T, e1, 0, 1, c->idmap(), nq, c->st);
    hec_ew(c->T, EW_FROM_MONT, m, pt->d, nullptr, 0, 0, 0, 1, c->idmap(), nq, c->st);
    hec_encrypt_finish(c->T, ct->d, v, e0, e1, m, c->d_pk, (size_t)(c->L + 1) * n, nq, c->st);
    c->release(buf);
    c->release(sm);
    HEC_TRY_HIP(hipGetLastError());
    *out = ct;
    return HEC_OK;
}
extern "C" hec_status ckks_encrypt(hec_ctx *c, const hec_pt *pt, uint64_t seed, hec_ct **out)
{
    return ckks_encrypt_idx(c, pt, seed, 0, out);
}

hec_status decrypt_slots(hec_ctx *c, const hec_ct *ct, double *z, size_t nz)
{
    // m = c0 + c1 s, back to coefficients, centered CRT and the decoding FFT
    // on the device; only the nz slot values come back
    const size_t n = c->n, nq = ct->level + 1;
    u64 *t = c->alloc(nq * n + n + 2 * n + c->N);
    if (!t) HEC_FAIL(HEC_ENOMEM, "decryption buffer");
    double *dm = (double *)(t + nq * n);
    double2 *work = (double2 *)(t + nq * n + n);
    double *dz = (double *)(t + nq * n + 3 * n);
    hec_ew(c->T, EW_MUL_MONT, t, ct->d + nq * n, c->d_sM, 0, 0, 0, 1, c->idmap(), nq, c->st);
    hec_ew(c->T, EW_ADD, t, t, ct->d, 0, 0, 0, 1, c->idmap(), nq, c->st);
    hec_ntt_inv(c->T, t, 0, 1, c->idmap(), nq, c->st);
    hec_crt_double(c->T, t, dm, (int)nq, c->d_crt_m, c->d_crt_inv, c->d_crt_invsh, c->st);
    hec_decode(dm, ct->scale, c->d_enc_root, c->d_enc_tw, work, dz, (u32)nz, c->logn, c->st);
    hipError_t e = hipSuccess;
    if (nz) e = hipMemcpyAsync(z, dz, nz * 8, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    c->release(t);
    if (e != hipSuccess) HEC_FAIL(HEC_EDEVICE, "decryption: %s", hipGetErrorString(e));
    return HEC_OK;
}

extern "C" hec_status ckks_decrypt(hec_ctx *c, const hec_ct *ct, double *z, size_t nz)
{
    if (!c || !ct || (nz && !z)) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (!c->have_keys) HEC_FAIL(HEC_ENOKEY, "no secret key");
    if (nz > c->N) HEC_FAIL(HEC_EINVAL, "more values than slots");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    return decrypt_slots(c, ct, z, nz);
}

// ---------------------------------------------------------------------------
// import / export
// ---------------------------------------------------------------------------
extern "C" hec_status ckks_ct_export(hec_ctx *c, const hec_ct *ct, uint64_t *coeff, uint32_t *level, double *scale)
{
    if (!c || !ct || !coeff) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    const size_t n = c->n, nq = ct->level + 1;
    u64 *t = c->alloc(2 * nq * n);
    if (!t) HEC_FAIL(HEC_ENOMEM, "export buffer");
    HEC_TRY_HIP(hipMemcpyAsync(t, ct->d, 2 * nq * n * 8, hipMemcpyDeviceToDevice, c->st));
    hec_ntt_inv(c->T, t, nq * n, 2, c->idmap(), nq, c->st);
    HEC_TRY_HIP(hipMemcpyAsync(coeff, t, 2 * nq * n * 8, hipMemcpyDeviceToHost, c->st));
    HEC_TRY_HIP(hipStreamSynchronize(c->st));
    c->release(t);
    if (level) *level = ct->level;
    if (scale) *scale = ct->scale;
    return HEC_OK;
}

extern "C" hec_status ckks_ct_import(hec_ctx *c, const uint64_t *coeff, uint32_t level, double scale, hec_ct **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !coeff) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (level > c->L) HEC_FAIL(HEC_ELEVEL, "level above L");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    const size_t n = c->n, nq = level + 1;
    for (size_t p = 0; p < 2; p++)
        for (size_t i = 0; i < nq; i++)
            for (size_t t = 0; t < n; t++)
                if (coeff[(p * nq + i) * n + t] >= c->mod[i]) HEC_FAIL(HEC_EINVAL, "residue not reduced");
    hec_ct *ct = ct_new(c, level, scale);
    if (!ct) HEC_FAIL(HEC_ENOMEM, "ciphertext allocation");
    HEC_TRY_HIP(hipMemcpyAsync(ct->d, coeff, 2 * nq * n * 8, hipMemcpyHostToDevice, c->st));
    hec_ntt_fwd(c->T, ct->d, nq * n, 2, c->idmap(), nq, c->st);
    HEC_TRY_HIP(hipStreamSynchronize(c->st));
    *out = ct;
    return HEC_OK;
}

// ---------------------------------------------------------------------------
// rotations (hybrid key switching)
// ---------------------------------------------------------------------------
// ModUp of c1 (hoisted once for all rotations of a ciphertext) of cnt
// ciphertexts at one level: D_i[j] = ModUp of digit j of ct i over Q_l and P,
// NTT form, at Dall + (i * beta + j) * (nq + k) * n.  One inverse NTT over all
// inputs, one base-conversion launch for all digits of all inputs (their own
// limbs copied), one forward NTT over everything: small launches leave most
// of the GPU idle, so batching ciphertexts pays.
hec_status ct_modup_many(hec_ctx *c, const std::vector<const hec_ct *> &cts, u64 **Dall)
{
    *Dall = nullptr;
    if (cts.empty()) return HEC_OK;
    const size_t n = c->n, cnt = cts.size();
    const uint32_t lvl = cts[0]->level, nq = lvl + 1, k = c->k, nqp = nq + k;
    for (auto *ct : cts)
        if (ct->level != lvl) HEC_FAIL(HEC_ELEVEL, "ModUp of ciphertexts at different levels");
    const uint32_t beta = (nq + c->alpha - 1) / c->alpha;
    u64 *cc = c->alloc(cnt * nq * n);
    u64 *D = c->alloc(cnt * beta * nqp * n);
    if (!cc || !D) {
        c->release(cc);
        c->release(D);
        HEC_FAIL(HEC_ENOMEM, "key-switch buffers");
    }
    // c1 to coefficients; every digit converted to Q_l and P with its own limbs
    // copied, then one forward NTT (the digit's own limbs come back to c1's values)
    // inputs at one stride from each other (a single one, or views into one
    // batch) go straight into the inverse NTT; others are copied first
    const ptrdiff_t stride = cnt > 1 ? cts[1]->d - cts[0]->d : 0;
    bool uniform = stride >= 0;
    for (size_t i = 1; i < cnt && uniform; i++) uniform = cts[i]->d == cts[0]->d + (ptrdiff_t)i * stride;
    if (!uniform || !hec_ntt_inv_from(c->T, cc, nq * n, cts[0]->d + nq * n, (size_t)stride, (int)cnt, c->idmap(),
                                      (int)nq, c->st)) {
        for (size_t i = 0; i < cnt; i++)
            HEC_TRY_HIP(
                hipMemcpyAsync(cc + i * nq * n, cts[i]->d + nq * n, nq * n * 8, hipMemcpyDeviceToDevice, c->st));
        hec_ntt_inv(c->T, cc, nq * n, (int)cnt, c->idmap(), nq, c->st);
    }
    uint32_t nout_max = 0, nin_max = 0;
    for (uint32_t j = 0; j < beta; j++) {
        nout_max = std::max(nout_max, c->h_modup[(size_t)lvl * c->dnum + j].nout);
        nin_max = std::max(nin_max, c->h_modup[(size_t)lvl * c->dnum + j].nin);
    }
    hec_bconv(c->T, c->d_modup + (size_t)lvl * c->dnum, 1, (int)beta, (int)nout_max, cc, D, nq * n,
              (size_t)nqp * n, (int)(cnt * beta), 1, c->st, (int)nin_max);
    hec_ntt_fwd(c->T, D, (size_t)nqp * n, (int)(cnt * beta), c->qpmap(lvl), (int)nqp, c->st);
    c->release(cc);
    *Dall = D;
    return HEC_OK;
}

hec_status ct_modup(hec_ctx *c, const hec_ct *ct, u64 **Dout) { return ct_modup_many(c, {ct}, Dout); }

const u64 *ones_qp(hec_ctx *c, uint32_t lvl)
{
    auto it = c->ones_qp.find(lvl);
    if (it != c->ones_qp.end()) return it->second;
    PoolScope ps(c, &c->pool);  // cached for the context's lifetime
    const size_t n = c->n, nqp = lvl + 1 + c->k;
    std::vector<u64> h(nqp * n);
    for (size_t l = 0; l < nqp; l++) {
        const u64 q = c->mod[l <= lvl ? l : c->L + 1 + (l - lvl - 1)];
        std::fill(h.begin() + l * n, h.begin() + (l + 1) * n, (u64)(((u128)1 << 64) % q));
    }
    u64 *d = c->alloc(nqp * n);
    if (!d) return nullptr;
    if (hipMemcpyAsync(d, h.data(), nqp * n * 8, hipMemcpyHostToDevice, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess) {
        c->release(d);
        return nullptr;
    }
    c->ones_qp[lvl] = d;
    return d;
}

// outs[i] = ModDown(E_i) for E_i = [2][nq+k][n] over Q_l and P (NTT form) at
// Eall + i * 2 (nq+k) n, all at one level; the P limbs of Eall are consumed.
// One launch per stage for all of them (combine in groups of HEC_KS_BATCH).
hec_status ct_moddown_many(hec_ctx *c, uint32_t lvl, u64 *Eall, const std::vector<hec_ct *> &outs,
                           const std::vector<std::array<const u64 *, 2>> *adds)
{
    if (outs.empty()) return HEC_OK;
    const size_t n = c->n, cnt = outs.size();
    const uint32_t nq = lvl + 1, k = c->k, nqp = nq + k;
    for (auto *o : outs)
        if (o->level != lvl) HEC_FAIL(HEC_ELEVEL, "ModDown output at another level");
    u64 *y = c->alloc(cnt * 2 * (size_t)nq * n);
    if (!y) HEC_FAIL(HEC_ENOMEM, "ModDown buffer");
    hec_ntt_inv(c->T, Eall + (size_t)nq * n, (size_t)nqp * n, (int)(2 * cnt), c->qpmap(lvl) + nq, k, c->st);
    hec_bconv(c->T, c->d_moddown + lvl, 0, 1, nq, Eall, y, (size_t)nqp * n, (size_t)nq * n, (int)(2 * cnt), 0,
              c->st, (int)c->k);
    const bool fused = c->logn == 16;  // the combine as the epilogue of the forward NTT's row pass
    if (!fused) hec_ntt_fwd(c->T, y, (size_t)nq * n, (int)(2 * cnt), c->qpmap(lvl), nq, c->st);
    for (size_t b0 = 0; b0 < cnt; b0 += HEC_KS_BATCH) {
        const size_t nb = std::min((size_t)HEC_KS_BATCH, cnt - b0);
        CombineBatch cb{};
        for (size_t r = 0; r < nb; r++) {
            cb.out[r] = outs[b0 + r]->d;
            cb.e[r] = Eall + (b0 + r) * 2 * (size_t)nqp * n;
            cb.y[r] = y + (b0 + r) * 2 * (size_t)nq * n;
            cb.g[r] = 1;
            if (adds) {
                cb.add[r][0] = (*adds)[b0 + r][0];
                cb.add[r][1] = (*adds)[b0 + r][1];
            }
        }
        if (!fused || !hec_ntt_fwd_moddown(c->T, y + b0 * 2 * (size_t)nq * n, (int)nb, (int)nq, (int)nqp, cb,
                                           c->d_lvl + lvl, c->qpmap(lvl), c->st))
            hec_moddown_combine(c->T, cb, (int)nb, nullptr, nq, nqp, c->d_lvl + lvl, c->qpmap(lvl), c->st);
    }
    c->release(y);
    HEC_TRY_HIP(hipGetLastError());
    return HEC_OK;
}

hec_status ct_moddown(hec_ctx *c, uint32_t lvl, u64 *E, hec_ct *out) { return ct_moddown_many(c, lvl, E, {out}); }

hec_status ct_rotate_hoisted(hec_ctx *c, const hec_ct *ct, const int32_t *steps, size_t cnt, hec_ct **outs,
                             const u64 *Dg)
{
    const size_t n = c->n;
    const uint32_t lvl = ct->level, nq = lvl + 1, k = c->k, nqp = nq + k;
    const uint32_t beta = (nq + c->alpha - 1) / c->alpha;
    std::vector<size_t> todo;
    for (size_t i = 0; i < cnt; i++) outs[i] = nullptr;
    for (size_t i = 0; i < cnt; i++) {
        uint32_t g = c->galois(steps[i]);
        if (g == 1) continue;
        if (!c->rotkeys.count(g)) HEC_FAIL(HEC_ENOKEY, "no rotation key for step %d", steps[i]);
        todo.push_back(i);
    }
    for (size_t i = 0; i < cnt; i++)
        if (c->galois(steps[i]) == 1) {
            outs[i] = ct_clone(c, ct);
            if (!outs[i]) HEC_FAIL(HEC_ENOMEM, "ciphertext allocation");
        }
    if (todo.empty()) return HEC_OK;
    // the digits: the caller's, or this call's own ModUp (released at the end)
    u64 *Down = nullptr;
    if (!Dg) HEC_CHECK(ct_modup(c, ct, &Down));
    const u64 *D = Dg ? Dg : Down;
    const u64 *c0 = ct->d;
    // key switch in batches; with more than one batch and ks_overlap, odd
    // batches run on the side stream (forked after the ModUp, joined at the
    // end), each stream with its own buffers, so that one batch's key switch
    // overlaps the other's ModDown; the residues do not depend on it
    const size_t kbn = (size_t)std::max(1, std::min((int)HEC_ROT_BATCH, hec_tune_params().ks_rot_batch));
    const size_t nb = (todo.size() + kbn - 1) / kbn;
    // (not while the stream is being captured into a graph: a recording
    // stays on the one stream it captures)
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (nb > 1 && hec_tune_params().ks_overlap) (void)hipStreamIsCapturing(c->st, &cap);
    const bool two = nb > 1 && hec_tune_params().ks_overlap && cap == hipStreamCaptureStatusNone;
    if (two) {
        hec_status f = side_stream(c);
        if (f == HEC_OK) {
            hipError_t e = hipEventRecord(c->ev_fork, c->st);
            if (e == hipSuccess) e = hipStreamWaitEvent(c->side, c->ev_fork, 0);
            if (e != hipSuccess) f = HEC_EDEVICE, hec_set_error("stream fork: %s", hipGetErrorString(e));
        }
        if (f != HEC_OK) {
            c->release(Down);
            for (size_t i = 0; i < cnt; i++) {
                ct_free(outs[i]);
                outs[i] = nullptr;
            }
            return f;
        }
    }
    const size_t emax = std::min(kbn, todo.size()) * 2 * nqp * n, ymax = std::min(kbn, todo.size()) * 2 * nq * n;
    u64 *E[2] = {c->alloc(emax), two ? c->alloc(emax) : nullptr};
    u64 *Y[2] = {c->alloc(ymax), two ? c->alloc(ymax) : nullptr};
    hec_status s = (!E[0] || !Y[0] || (two && (!E[1] || !Y[1]))) ? HEC_ENOMEM : HEC_OK;
    if (s != HEC_OK) hec_set_error("key-switch buffers");
    for (size_t b0 = 0, bi = 0; b0 < todo.size() && s == HEC_OK; b0 += kbn, bi++) {
        const int R = (int)std::min(kbn, todo.size() - b0);
        const int side = two ? (int)(bi & 1) : 0;
        hipStream_t st = side ? c->side : c->st;
        u64 *e = E[side], *y = Y[side];
        KsBatch kb{};
        CombineBatch cb{};
        for (int r = 0; r < R && s == HEC_OK; r++) {
            size_t i = todo[b0 + r];
            uint32_t g = c->galois(steps[i]);
            hec_ct *o = ct_new(c, lvl, ct->scale);
            if (!o) {
                s = HEC_ENOMEM;
                hec_set_error("ciphertext allocation");
                break;
            }
            outs[i] = o;
            kb.key[r] = c->rotkeys[g];
            kb.out[r] = e + (size_t)r * 2 * nqp * n;
            kb.g[r] = g;
            kb.c0[r] = c0;  // P * sigma_g(c0) folded into the key-switch product
            cb.out[r] = o->d;
            cb.e[r] = kb.out[r];
            cb.y[r] = y + (size_t)r * 2 * nq * n;
            cb.g[r] = g;
        }
        if (s != HEC_OK) break;
        hec_ks_inner(c->T, kb, R, D, beta, nqp, c->qpmap(lvl), c->NLK, st, c->d_pmodq_m, (int)nq);
        c->ks_count += (uint64_t)R;
        // ModDown: INTT of the P limbs, P -> Q_l conversion, NTT, combine (the
        // combine fused into the NTT's last pass where the ring allows)
        hec_ntt_inv(c->T, e + (size_t)nq * n, (size_t)nqp * n, 2 * R, c->qpmap(lvl) + nq, k, st);
        hec_bconv(c->T, c->d_moddown + lvl, 0, 1, nq, e, y, (size_t)nqp * n, (size_t)nq * n, 2 * R, 0, st, (int)c->k);
        // (cb.c0 stays null: sigma_g(c0) is already in e)
        if (!hec_ntt_fwd_moddown(c->T, y, R, (int)nq, (int)nqp, cb, c->d_lvl + lvl, c->qpmap(lvl), st)) {
            hec_ntt_fwd(c->T, y, (size_t)nq * n, 2 * R, c->qpmap(lvl), nq, st);
            hec_moddown_combine(c->T, cb, R, nullptr, nq, nqp, c->d_lvl + lvl, c->qpmap(lvl), st);
        }
    }
    if (two) {
        // join: the main stream waits for the side stream's batches before
        // anything after this call (and before the buffers are reused)
        hipError_t e1 = hipEventRecord(c->ev_join, c->side);
        hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(c->st, c->ev_join, 0) : e1;
        if (e2 != hipSuccess && s == HEC_OK) {
            s = HEC_EDEVICE;
            hec_set_error("stream join: %s", hipGetErrorString(e2));
        }
    }
    for (int i = 0; i < 2; i++) {
        c->release(E[i]);
        c->release(Y[i]);
    }
    if (s != HEC_OK) {
        c->release(Down);
        for (size_t i = 0; i < cnt; i++) {
            ct_free(outs[i]);
            outs[i] = nullptr;
        }
        return s;
    }
    c->release(Down);
    HEC_TRY_HIP(hipGetLastError());
    return HEC_OK;
}

static void free_all_cts(std::vector<hec_ct *> &v)
{
    for (auto *&p : v) {
        ct_free(p);
        p = nullptr;
    }
}

hec_status ct_rotate_many(hec_ctx *c, const std::vector<const hec_ct *> &cts, int32_t step, std::vector<hec_ct *> &outs)
{
    outs.assign(cts.size(), nullptr);
    if (cts.empty()) return HEC_OK;
    const size_t n = c->n;
    const uint32_t lvl = cts[0]->level, nq = lvl + 1, k = c->k, nqp = nq + k;
    const uint32_t beta = (nq + c->alpha - 1) / c->alpha;
    for (auto *ct : cts)
        if (ct->level != lvl) HEC_FAIL(HEC_ELEVEL, "batched rotation of ciphertexts at different levels");
    const uint32_t g = c->galois(step);
    if (g == 1) {
        for (size_t i = 0; i < cts.size(); i++)
            if (!(outs[i] = ct_clone(c, cts[i]))) {
                free_all_cts(outs);
                HEC_FAIL(HEC_ENOMEM, "ciphertext allocation");
            }
        return HEC_OK;
    }
    if (!c->rotkeys.count(g)) HEC_FAIL(HEC_ENOKEY, "no rotation key for step %d", step);
    u64 *Dall = nullptr;
    HEC_CHECK(ct_modup_many(c, cts, &Dall));
    hec_status s = HEC_OK;
    for (size_t b0 = 0; b0 < cts.size() && s == HEC_OK; b0 += HEC_KS_BATCH) {
        const int R = (int)std::min((size_t)HEC_KS_BATCH, cts.size() - b0);
        u64 *e = c->alloc((size_t)R * 2 * nqp * n);
        u64 *y = c->alloc((size_t)R * 2 * nq * n);
        KsBatch kb{};
        CombineBatch cb{};
        for (int r = 0; r < R && e && y; r++) {
            const size_t i = b0 + r;
            if (!(outs[i] = ct_new(c, lvl, cts[i]->scale))) break;
            kb.key[r] = c->rotkeys[g];
            kb.out[r] = e + (size_t)r * 2 * nqp * n;
            kb.D[r] = Dall + i * beta * (size_t)nqp * n;
            kb.g[r] = g;
            cb.out[r] = outs[i]->d;
            cb.e[r] = kb.out[r];
            cb.y[r] = y + (size_t)r * 2 * nq * n;
            cb.c0[r] = cts[i]->d;
            cb.g[r] = g;
        }
        bool ok = e && y;
        for (int r = 0; r < R; r++) ok = ok && outs[b0 + r];
        if (!ok) {
            s = HEC_ENOMEM;
            hec_set_error("key-switch buffers");
        } else {
            hec_ks_inner(c->T, kb, R, nullptr, beta, nqp, c->qpmap(lvl), c->NLK, c->st);
            c->ks_count += (uint64_t)R;
            hec_ntt_inv(c->T, e + (size_t)nq * n, (size_t)nqp * n, 2 * R, c->qpmap(lvl) + nq, k, c->st);
            hec_bconv(c->T, c->d_moddown + lvl, 0, 1, nq, e, y, (size_t)nqp * n, (size_t)nq * n, 2 * R, 0, c->st, (int)c->k);
            if (!hec_ntt_fwd_moddown(c->T, y, R, (int)nq, (int)nqp, cb, c->d_lvl + lvl, c->qpmap(lvl), c->st)) {
                hec_ntt_fwd(c->T, y, (size_t)nq * n, 2 * R, c->qpmap(lvl), nq, c->st);
                hec_moddown_combine(c->T, cb, R, nullptr, nq, nqp, c->d_lvl + lvl, c->qpmap(lvl), c->st);
            }
        }
        c->release(e);
        c->release(y);
    }
    c->release(Dall);
    if (s == HEC_OK && hipGetLastError() != hipSuccess) s = HEC_EDEVICE, hec_set_error("batched rotation launch");
    if (s != HEC_OK) free_all_cts(outs);
    return s;
}

// Key-stationary hoisted rotations of several ciphertexts at one level: every
// input takes one ModUp (all in one set of launches), then the nonzero amounts
// go through the key switch in batches of `batch` (<= HEC_KS_BATCH), each key
// read once for all inputs of its batch (k_ks_inner_multi), and the ModDowns of
// a batch's rotations share one set of NTT and base-conversion launches.
// want[a] has bit u set when input u needs amount a.  sink(a0, na, rots) gets
// the rotations of amounts a0 .. a0+na-1 as rots[(a - a0) * S + u] (null
// where not wanted), valid until it returns; they equal ct_rotate_hoisted's bit
// for bit (same ModUp, the same inner products and reductions, same ModDown).
hec_status ct_rotate_multi(hec_ctx *c, const std::vector<const hec_ct *> &ins, const std::vector<int32_t> &amounts,
                           const std::vector<uint64_t> &want, size_t batch, const RotSink &sink)
{
    const size_t S = ins.size();
    if (!S || amounts.empty()) return HEC_OK;
    if (S > HEC_MULTI_MAX_INPUTS) HEC_FAIL(HEC_EINVAL, "more than %d inputs in a key-stationary batch",
                                           HEC_MULTI_MAX_INPUTS);
    if (want.size() != amounts.size()) HEC_FAIL(HEC_EINVAL, "one input mask per amount");
    batch = std::max<size_t>(1, std::min<size_t>(batch, HEC_KS_BATCH));
    const size_t n = c->n;
    const uint32_t lvl = ins[0]->level, nq = lvl + 1, k = c->k, nqp = nq + k;
    const uint32_t beta = (nq + c->alpha - 1) / c->alpha;
    for (int32_t a : amounts) {
        const uint32_t g = c->galois(a);
        if (g == 1) HEC_FAIL(HEC_EINVAL, "zero rotation in a key-stationary batch");
        if (!c->rotkeys.count(g)) HEC_FAIL(HEC_ENOKEY, "no rotation key for step %d", a);
    }
    u64 *Dall = nullptr;
    HEC_CHECK(ct_modup_many(c, ins, &Dall));
    const size_t dstride = (size_t)beta * nqp * n, estride = 2ull * nqp * n, ystride = 2ull * nq * n;
    hec_status s = HEC_OK;
    for (size_t a0 = 0; a0 < amounts.size() && s == HEC_OK; a0 += batch) {
        const size_t na = std::min(batch, amounts.size() - a0), R = na * S;
        u64 *e = c->alloc(R * estride), *y = c->alloc(R * ystride), *ro = c->alloc(R * ystride);
        if (!e || !y || !ro) {
            c->release(e);
            c->release(y);
            c->release(ro);
            s = HEC_ENOMEM;
            hec_set_error("key-stationary rotation buffers");
            break;
        }
        KsMulti kb{};
        for (size_t t = 0; t < na; t++) {
            const uint32_t g = c->galois(amounts[a0 + t]);
            kb.key[t] = c->rotkeys[g];
            kb.out[t] = e + t * S * estride;
            kb.mask[t] = want[a0 + t];
            kb.g[t] = g;
            c->ks_count += (uint64_t)__builtin_popcountll(want[a0 + t]);
        }
        if (!hec_ks_inner_multi(c->T, kb, (int)na, Dall, dstride, (int)S, estride, (int)beta, (int)nqp,
                                c->qpmap(lvl), (int)c->NLK, c->st)) {
            s = HEC_EINVAL;
            hec_set_error("key-stationary key switch launch");
        }
        // ModDown of every slot of the batch (slots not wanted carry unused
        // values); the combine as the epilogue of the forward NTT where the
        // ring allows, in groups of HEC_KS_BATCH consecutive slots
        const bool fused = c->logn == 16;
        if (s == HEC_OK) {
            hec_ntt_inv(c->T, e + (size_t)nq * n, (size_t)nqp * n, (int)(2 * R), c->qpmap(lvl) + nq, k, c->st);
            hec_bconv(c->T, c->d_moddown + lvl, 0, 1, nq, e, y, (size_t)nqp * n, (size_t)nq * n, (int)(2 * R), 0,
                      c->st, (int)c->k);
            if (!fused) hec_ntt_fwd(c->T, y, (size_t)nq * n, (int)(2 * R), c->qpmap(lvl), nq, c->st);
        }
        std::vector<hec_ct> cts(R);
        std::vector<hec_ct *> rots(R, nullptr);
        for (size_t r0 = 0; r0 < R && s == HEC_OK; r0 += HEC_KS_BATCH) {
            const size_t nr = std::min((size_t)HEC_KS_BATCH, R - r0);
            CombineBatch cb{};
            int nb = 0;
            for (size_t r = r0; r < r0 + nr; r++) {
                const size_t t = r / S, u = r % S;
                const int slot = fused ? (int)(r - r0) : nb;
                if (!((want[a0 + t] >> u) & 1)) continue;
                cts[r].ctx = c;
                cts[r].level = lvl;
                cts[r].scale = ins[u]->scale;
                cts[r].d = ro + r * ystride;
                rots[r] = &cts[r];
                cb.out[slot] = cts[r].d;
                cb.e[slot] = e + r * estride;
                cb.y[slot] = y + r * ystride;
                cb.c0[slot] = ins[u]->d;
                cb.g[slot] = kb.g[t];
                nb++;
            }
            if (fused)
                hec_ntt_fwd_moddown(c->T, y + r0 * ystride, (int)nr, (int)nq, (int)nqp, cb, c->d_lvl + lvl,
                                    c->qpmap(lvl), c->st);
            else if (nb)
                hec_moddown_combine(c->T, cb, nb, nullptr, nq, nqp, c->d_lvl + lvl, c->qpmap(lvl), c->st);
        }
        if (s == HEC_OK && hipGetLastError() != hipSuccess) s = HEC_EDEVICE, hec_set_error("key-stationary launch");
        if (s == HEC_OK) s = sink(a0, na, rots);
        c->release(e);
        c->release(y);
        c->release(ro);
    }
    c->release(Dall);
    return s;
}

extern "C" hec_status ckks_rotate_hoisted(hec_ctx *c, const hec_ct *ct, const int32_t *steps, size_t cnt,
                                          hec_ct **outs)
{
    if (!c || !ct || (cnt && (!steps || !outs))) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    hec_status s = ct_rotate_hoisted(c, ct, steps, cnt, outs);
    if (s != HEC_OK)
        for (size_t i = 0; i < cnt; i++) {
            ct_free(outs[i]);
            outs[i] = nullptr;
        }
    return s;
}

extern "C" hec_status ckks_rotate(hec_ctx *c, const hec_ct *ct, int32_t step, hec_ct **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    return ckks_rotate_hoisted(c, ct, &step, 1, out);
}

// The rotation of ckks_rotate with every temporary in the device's scratch
// array: c1 to coefficients, ModUp of its digits, key-switch inner product,
// ModDown and the sigma_g(c0) term, the same launches (hence the same bits)
// as ckks_rotate; nothing allocated, freed or synchronized.
extern "C" hec_status ckks_rotate_noalloc(hec_ctx *c, const hec_ct *in, int32_t step, hec_ct *out)
{
    if (!c || !in || !out) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (in->ctx != c || out->ctx != c) HEC_FAIL(HEC_EINVAL, "ciphertext of another context");
    if (out == in || out->d == in->d) HEC_FAIL(HEC_EINVAL, "out must not be the input");
    if (out->level != in->level) HEC_FAIL(HEC_ELEVEL, "out is at level %u, the input at %u", out->level, in->level);
    const size_t n = c->n;
    const uint32_t lvl = in->level, nq = lvl + 1, k = c->k, nqp = nq + k;
    const uint32_t beta = (nq + c->alpha - 1) / c->alpha;
    const uint32_t g = c->galois(step);
    HEC_TRY_HIP(hipSetDevice(c->dev));
    if (g == 1) {
        HEC_TRY_HIP(hipMemcpyAsync(out->d, in->d, 2 * (size_t)nq * n * 8, hipMemcpyDeviceToDevice, c->st));
        out->scale = in->scale;
        return HEC_OK;
    }
    auto key = c->rotkeys.find(g);
    if (key == c->rotkeys.end()) HEC_FAIL(HEC_ENOKEY, "no rotation key for step %d", step);
    // c1 in coefficient form, the ModUp digits, the key-switch product and the
    // P -> Q conversion, one after the other in the scratch array
    const size_t words = n * ((size_t)nq + (size_t)beta * nqp + 2ull * nqp + 2ull * nq);
    if (words * 8 > HEC_NOALLOC_SCRATCH_BYTES)
        HEC_FAIL(HEC_EINVAL, "rotation at level %u needs %zu MiB of scratch, the limit is %llu MiB", lvl,
                 (words * 8) >> 20, (unsigned long long)(HEC_NOALLOC_SCRATCH_BYTES >> 20));
    u64 *const sp = g_scratch_ptr[c->dev];
    if (!sp) HEC_FAIL(HEC_EDEVICE, "scratch not resolved on device %d", c->dev);
    u64 *cc = sp, *D = cc + (size_t)nq * n, *e = D + (size_t)beta * nqp * n, *y = e + 2ull * nqp * n;
    if (!hec_ntt_inv_from(c->T, cc, nq * n, in->d + (size_t)nq * n, 0, 1, c->idmap(), (int)nq, c->st)) {
        HEC_TRY_HIP(hipMemcpyAsync(cc, in->d + (size_t)nq * n, (size_t)nq * n * 8, hipMemcpyDeviceToDevice, c->st));
        hec_ntt_inv(c->T, cc, nq * n, 1, c->idmap(), nq, c->st);
    }
    uint32_t nout_max = 0, nin_max = 0;
    for (uint32_t j = 0; j < beta; j++) {
        nout_max = std::max(nout_max, c->h_modup[(size_t)lvl * c->dnum + j].nout);
        nin_max = std::max(nin_max, c->h_modup[(size_t)lvl * c->dnum + j].nin);
    }
    hec_bconv(c->T, c->d_modup + (size_t)lvl * c->dnum, 1, (int)beta, (int)nout_max, cc, D, nq * n, (size_t)nqp * n,
              (int)beta, 1, c->st, (int)nin_max);
    hec_ntt_fwd(c->T, D, (size_t)nqp * n, (int)beta, c->qpmap(lvl), (int)nqp, c->st);
    KsBatch kb{};
    kb.key[0] = key->second;
    kb.out[0] = e;
    kb.g[0] = g;
    hec_ks_inner(c->T, kb, 1, D, beta, nqp, c->qpmap(lvl), c->NLK, c->st);
    c->ks_count += 1;
    hec_ntt_inv(c->T, e + (size_t)nq * n, (size_t)nqp * n, 2, c->qpmap(lvl) + nq, k, c->st);
    hec_bconv(c->T, c->d_moddown + lvl, 0, 1, nq, e, y, (size_t)nqp * n, (size_t)nq * n, 2, 0, c->st, (int)c->k);
    CombineBatch cb{};
    cb.out[0] = out->d;
    cb.e[0] = e;
    cb.y[0] = y;
    cb.c0[0] = in->d;
    cb.g[0] = g;
    if (!hec_ntt_fwd_moddown(c->T, y, 1, (int)nq, (int)nqp, cb, c->d_lvl + lvl, c->qpmap(lvl), c->st)) {
        hec_ntt_fwd(c->T, y, (size_t)nq * n, 2, c->qpmap(lvl), nq, c->st);
        hec_moddown_combine(c->T, cb, 1, in->d, nq, nqp, c->d_lvl + lvl, c->qpmap(lvl), c->st);
    }
    HEC_TRY_HIP(hipGetLastError());
    out->scale = in->scale;
    return HEC_OK;
}

// ---------------------------------------------------------------------------
// rescale, products, sums
// ---------------------------------------------------------------------------
// npolys polynomials [npolys][l+1][n] at level l divided by q_l: *d replaced
// by [npolys][l][n] (the old buffer released)
hec_status rescale_polys(hec_ctx *c, u64 **d, uint32_t l, int npolys)
{
    if (l == 0) HEC_FAIL(HEC_ELEVEL, "cannot rescale at level 0");
    const size_t n = c->n, np = (size_t)npolys;
    const uint32_t nq = l + 1;
    u64 *last = c->alloc(np * n), *tmp = c->alloc(np * l * n), *o = c->alloc(np * l * n);
    if (!last || !tmp || !o) {
        c->release(last);
        c->release(tmp);
        c->release(o);
        HEC_FAIL(HEC_ENOMEM, "rescale buffers");
    }
    if (!hec_ntt_inv_from(c->T, last, n, *d + (size_t)l * n, (size_t)nq * n, npolys, c->idmap() + l, 1, c->st)) {
        hec_copy_limbs(last, *d + (size_t)l * n, n, (size_t)nq * n, npolys, n, c->st);
        hec_ntt_inv(c->T, last, n, npolys, c->idmap() + l, 1, c->st);
    }
    // (c_i - [centered last]_{q_i}) * q_l^-1: the reduction folded into the
    // forward NTT's loads and the last step into its stores where the ring allows
    const RescaleFuse f{last, n, *d, (size_t)nq * n, o, (size_t)l * n, c->d_lvl + l, l};
    if (!hec_ntt_fwd_rescale(c->T, tmp, npolys, c->idmap(), f, c->st)) {
        hec_rescale_spread(c->T, last, tmp, n, (size_t)l * n, npolys, l, c->st);
        hec_ntt_fwd(c->T, tmp, (size_t)l * n, npolys, c->idmap(), l, c->st);
        hec_rescale_finish(c->T, o, *d, tmp, (size_t)l * n, (size_t)nq * n, (size_t)l * n, npolys, l, c->d_lvl + l,
                           c->st);
    }
    c->release(last);
    c->release(tmp);
    c->release(*d);
    *d = o;
    HEC_TRY_HIP(hipGetLastError());
    return HEC_OK;
}

hec_status ct_rescale(hec_ctx *c, hec_ct *ct)
{
    HEC_CHECK(rescale_polys(c, &ct->d, ct->level, 2));
    ct->scale /= (double)c->mod[ct->level];
    ct->level -= 1;
    return HEC_OK;
}

extern "C" hec_status ckks_rescale(hec_ctx *c, hec_ct *ct)
{
    if (!c || !ct) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    return ct_rescale(c, ct);
}

hec_status ct_mac_pt(hec_ctx *c, hec_ct *acc, const hec_ct *ct, const hec_pt *pt, bool first)
{
    if (ct->level != pt->level || acc->level != ct->level) HEC_FAIL(HEC_ELEVEL, "level mismatch in pt product");
    const size_t n = c->n, nq = ct->level + 1;
    hec_ew(c->T, first ? EW_MUL_MONT : EW_MAC_MONT, acc->d, ct->d, pt->d, nq * n, nq * n, 0, 2, c->idmap(), nq,
           c->st);
    if (first) acc->scale = ct->scale * pt->scale;
    return HEC_OK;
}

hec_status ct_add_inplace(hec_ctx *c, hec_ct *acc, const hec_ct *b)
{
    if (acc->level != b->level) HEC_FAIL(HEC_ELEVEL, "level mismatch in addition");
    if (acc->scale != b->scale) HEC_FAIL(HEC_ESCALE, "scale mismatch in addition");
    const size_t n = c->n, nq = acc->level + 1;
    hec_ew(c->T, EW_ADD, acc->d, acc->d, b->d, nq * n, nq * n, nq * n, 2, c->idmap(), nq, c->st);
    return HEC_OK;
}

extern "C" hec_status ckks_mul_pt(hec_ctx *c, const hec_ct *ct, const hec_pt *pt, hec_ct **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !ct || !pt) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (ct->level != pt->level) HEC_FAIL(HEC_ELEVEL, "level mismatch");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    hec_ct *o = ct_new(c, ct->level, ct->scale * pt->scale);
    if (!o) HEC_FAIL(HEC_ENOMEM, "ciphertext allocation");
    hec_status s = ct_mac_pt(c, o, ct, pt, true);
    if (s != HEC_OK) { ct_free(o); return s; }
    *out = o;
    return HEC_OK;
}

extern "C" hec_status ckks_add(hec_ctx *c, const hec_ct *a, const hec_ct *b, hec_ct **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !a || !b) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (a->level != b->level) HEC_FAIL(HEC_ELEVEL, "level mismatch");
    if (a->scale != b->scale) HEC_FAIL(HEC_ESCALE, "scale mismatch");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    hec_ct *o = ct_clone(c, a);
    if (!o) HEC_FAIL(HEC_ENOMEM, "ciphertext allocation");
    hec_status s = ct_add_inplace(c, o, b);
    if (s != HEC_OK) { ct_free(o); return s; }
    *out = o;
    return HEC_OK;
}

// ---------------------------------------------------------------------------
// diagnostics
// ---------------------------------------------------------------------------
extern "C" hec_status hec_prof_start(hec_ctx *c, const char *kernel)
{
    if (!c || !kernel) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    HEC_TRY_HIP(hipStreamSynchronize(c->st));
    hec_prof_select(kernel);
    return HEC_OK;
}

extern "C" uint64_t hec_prof_launches(const char *kernel) { return kernel ? hec_prof_count(kernel) : 0; }

extern "C" hec_status hec_probe_stream(hec_ctx *c, int nread, int nwrite, uint64_t words, int reps,
                                       double *us_per_launch)
{
    if (!c || !us_per_launch) HEC_FAIL(HEC_EINVAL, "NULL argument");
    if (nread < 1 || nread > HEC_PROBE_MAX_READ || nwrite < 1 || nwrite > HEC_PROBE_MAX_WRITE)
        HEC_FAIL(HEC_EINVAL, "streams: 1..%d read, 1..%d written", HEC_PROBE_MAX_READ, HEC_PROBE_MAX_WRITE);
    if (words < 256 || words > (1ull << 32) || reps < 1 || reps > 10000) HEC_FAIL(HEC_EINVAL, "words or reps out of range");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    HEC_TRY_HIP(hipStreamSynchronize(c->st));
    u64 *in = nullptr, *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hec_status st = HEC_OK;
    float ms = 0;
    if (hipMalloc(&in, (size_t)nread * words * 8) != hipSuccess || hipMalloc(&out, (size_t)nwrite * words * 8) != hipSuccess) {
        (void)hipGetLastError();
        hec_set_error("probe buffers (%llu bytes)", (unsigned long long)((nread + nwrite) * words * 8));
        st = HEC_ENOMEM;
        goto done;
    }
    if (hipMemsetAsync(in, 1, (size_t)nread * words * 8, c->st) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        hec_set_error("probe set-up failed");
        st = HEC_EDEVICE;
        goto done;
    }
    hec_probe_stream(in, out, words, nread, nwrite, c->st);  // warm-up
    (void)hipEventRecord(e0, c->st);
    for (int i = 0; i < reps; i++) hec_probe_stream(in, out, words, nread, nwrite, c->st);
    (void)hipEventRecord(e1, c->st);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
        hipGetLastError() != hipSuccess) {
        hec_set_error("probe launch failed");
        st = HEC_EDEVICE;
        goto done;
    }
    *us_per_launch = ms * 1e3 / reps;
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (in) (void)hipFree(in);
    if (out) (void)hipFree(out);
    return st;
}

extern "C" hec_status hec_prof_stop(hec_ctx *c, uint64_t *launches, uint64_t *units, double *total_ms)
{
    if (!c || !launches || !units || !total_ms) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_TRY_HIP(hipSetDevice(c->dev));
    HEC_TRY_HIP(hipStreamSynchronize(c->st));
    if (hec_prof_collect(launches, units, total_ms) != 0) HEC_FAIL(HEC_EDEVICE, "event timing failed");
    hec_prof_select(nullptr);
    return HEC_OK;
}

// ---------------------------------------------------------------------------
// ciphertext products (tensor product + relinearization) and constants
// ---------------------------------------------------------------------------
// a * b = (d0, d1, d2) = (a0 b0, a0 b1 + a1 b0, a1 b1); d2 (a term in s^2) is
// switched to s with the relinearization key: ModUp(d2), inner product with
// the key over Q_l and P, ModDown, added to (d0, d1).  Scale a.scale * b.scale.
hec_status ct_mul(hec_ctx *c, const hec_ct *a, const hec_ct *b, hec_ct **out)
{
    *out = nullptr;
    if (a->level != b->level) HEC_FAIL(HEC_ELEVEL, "level mismatch in ciphertext product");
    const u64 *rlk = nullptr;
    HEC_CHECK(relin_key(c, &rlk));
    const size_t n = c->n;
    const uint32_t lvl = a->level, nq = lvl + 1, nqp = nq + c->k;
    const uint32_t beta = (nq + c->alpha - 1) / c->alpha;
    const size_t P = (size_t)nq * n;
    // t = [d0][d2][d1]: a ciphertext view (d0, d2) whose second polynomial is the one ModUp reads
    u64 *t = c->alloc(3 * P), *E = c->alloc(2 * (size_t)nqp * n);
    hec_ct *o = ct_new(c, lvl, a->scale * b->scale);
    if (!t || !E || !o) {
        c->release(t);
        c->release(E);
        ct_free(o);
        HEC_FAIL(HEC_ENOMEM, "ciphertext product buffers");
    }
    hec_tensor(c->T, t, a->d, b->d, (int)nq, 1, c->st);
    hec_ct view;
    view.ctx = c;
    view.level = lvl;
    view.d = t;
    u64 *D = nullptr;
    hec_status s = ct_modup(c, &view, &D);
    if (s == HEC_OK) {
        KsBatch kb{};
        kb.key[0] = rlk;
        kb.out[0] = E;
        kb.g[0] = 1;
        hec_ks_inner(c->T, kb, 1, D, (int)beta, (int)nqp, c->qpmap(lvl), (int)c->NLK, c->st);
        c->ks_count += 1;
        // ModDown of the key-switched d2 plus (d0, d1), which sit at t and t + 2P
        const std::vector<std::array<const u64 *, 2>> adds{{t, t + 2 * P}};
        s = ct_moddown_many(c, lvl, E, {o}, &adds);
        if (s == HEC_OK && hipGetLastError() != hipSuccess)
            s = HEC_EDEVICE, hec_set_error("ciphertext product launch failed");
    }
    c->release(D);
    c->release(t);
    c->release(E);
    if (s != HEC_OK) {
        ct_free(o);
        return s;
    }
    *out = o;
    return HEC_OK;
}

// A constant in every slot encodes as the constant polynomial
// round_half_away(value * scale), the product of the two doubles taken
// exactly (53-bit mantissas multiplied in 128 bits).
hec_status const_coeff(double value, double scale, int64_t *r)
{
    if (!std::isfinite(value) || !std::isfinite(scale)) HEC_FAIL(HEC_EINVAL, "constant or scale not finite");
    *r = 0;
    if (value == 0.0 || scale == 0.0) return HEC_OK;
    int ea, eb;
    double fa = std::frexp(std::fabs(value), &ea), fb = std::frexp(std::fabs(scale), &eb);
    const u128 P = (u128)(uint64_t)std::ldexp(fa, 53) * (u128)(uint64_t)std::ldexp(fb, 53);
    const int e = ea + eb - 106;  // |value * scale| = P * 2^e
    u128 m;
    if (e >= 0) {
        if (e >= 62 || (P >> (62 - e)) != 0) HEC_FAIL(HEC_EINVAL, "constant exceeds 2^62");
        m = P << e;
    } else if (-e >= 120) {
        m = 0;
    } else {
        const int s = -e;
        m = (P + ((u128)1 << (s - 1))) >> s;
    }
    if (m >= ((u128)1 << 62)) HEC_FAIL(HEC_EINVAL, "constant exceeds 2^62");
    const bool neg = (value < 0) != (scale < 0);
    *r = neg ? -(int64_t)m : (int64_t)m;
    return HEC_OK;
}

void scalar_arg(const hec_ctx *c, int64_t r, uint32_t nlimbs, ScalarArg &sa)
{
    for (uint32_t l = 0; l < nlimbs; l++) {
        const u64 q = c->mod[l];
        u64 v = (u64)(r >= 0 ? (u128)r % q : (q - (u64)((u128)(-(r + 1)) % q) - 1));
        sa.v[l] = v;
        sa.vsh[l] = (u64)(((u128)v << 64) / q);
    }
}

hec_status ct_mul_const(hec_ctx *c, const hec_ct *a, double value, double pscale, hec_ct **out)
{
    return ct_mul_const_at(c, a, a->level, value, pscale, out);
}

// a's first level+1 limbs (a dropped to `level`) times the constant
hec_status ct_mul_const_at(hec_ctx *c, const hec_ct *a, uint32_t level, double value, double pscale, hec_ct **out)
{
    *out = nullptr;
    if (level > a->level) HEC_FAIL(HEC_ELEVEL, "cannot raise a level");
    int64_t r;
    HEC_CHECK(const_coeff(value, pscale, &r));
    hec_ct *o = ct_new(c, level, a->scale * pscale);
    if (!o) HEC_FAIL(HEC_ENOMEM, "ciphertext allocation");
    ScalarArg sa;
    scalar_arg(c, r, level + 1, sa);
    hec_scalar(c->T, SC_MUL, o->d, a->d, (size_t)(level + 1) * c->n, (size_t)(a->level + 1) * c->n, 2,
               (int)level + 1, 0, sa, c->st);
    *out = o;
    return HEC_OK;
}

hec_status ct_add_const(hec_ctx *c, const hec_ct *a, double value, double scale, hec_ct **out)
{
    *out = nullptr;
    int64_t r;
    HEC_CHECK(const_coeff(value, scale, &r));
    hec_ct *o = ct_new(c, a->level, a->scale);
    if (!o) HEC_FAIL(HEC_ENOMEM, "ciphertext allocation");
    ScalarArg sa;
    scalar_arg(c, r, a->level + 1, sa);
    const size_t P = (size_t)(a->level + 1) * c->n;
    hec_scalar(c->T, SC_ADD, o->d, a->d, P, P, 2, (int)a->level + 1, 0, sa, c->st);
    *out = o;
    return HEC_OK;
}

hec_status ct_sub(hec_ctx *c, const hec_ct *a, const hec_ct *b, hec_ct **out)
{
    *out = nullptr;
    if (a->level != b->level) HEC_FAIL(HEC_ELEVEL, "level mismatch in subtraction");
    if (a->scale != b->scale) HEC_FAIL(HEC_ESCALE, "scale mismatch in subtraction");
    hec_ct *o = ct_new(c, a->level, a->scale);
    if (!o) HEC_FAIL(HEC_ENOMEM, "ciphertext allocation");
    const size_t P = (size_t)(a->level + 1) * c->n;
    hec_ew(c->T, EW_SUB, o->d, a->d, b->d, P, P, P, 2, c->idmap(), (int)a->level + 1, c->st);
    *out = o;
    return HEC_OK;
}

// the first level+1 limbs of both polynomials (modulus dropped, scale kept)
hec_status ct_drop(hec_ctx *c, const hec_ct *a, uint32_t level, hec_ct **out)
{
    *out = nullptr;
    if (level > a->level) HEC_FAIL(HEC_ELEVEL, "cannot raise a level");
    hec_ct *o = ct_new(c, level, a->scale);
    if (!o) HEC_FAIL(HEC_ENOMEM, "ciphertext allocation");
    hec_copy_limbs(o->d, a->d, (size_t)(level + 1) * c->n, (size_t)(a->level + 1) * c->n, 2,
                   (size_t)(level + 1) * c->n, c->st);
    *out = o;
    return HEC_OK;
}

#define HEC_ABI_OUT1(call)                                                                                         \
    do {                                                                                                           \
        HEC_TRY_HIP(hipSetDevice(c->dev));                                                                         \
        hec_status s_ = (call);                                                                                    \
        if (s_ == HEC_OK && hipGetLastError() != hipSuccess) {                                                     \
            ct_free(*out);                                                                                         \
            *out = nullptr;                                                                                        \
            HEC_FAIL(HEC_EDEVICE, "kernel launch failed");                                                         \
        }                                                                                                          \
        return s_;                                                                                                 \
    } while (0)

extern "C" hec_status ckks_mul(hec_ctx *c, const hec_ct *a, const hec_ct *b, hec_ct **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !a || !b) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_ABI_OUT1(ct_mul(c, a, b, out));
}

extern "C" hec_status ckks_mul_const(hec_ctx *c, const hec_ct *a, double value, double pscale, hec_ct **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !a) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_ABI_OUT1(ct_mul_const(c, a, value, pscale, out));
}

extern "C" hec_status ckks_add_const(hec_ctx *c, const hec_ct *a, double value, hec_ct **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !a) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_ABI_OUT1(ct_add_const(c, a, value, a->scale, out));
}

extern "C" hec_status ckks_sub(hec_ctx *c, const hec_ct *a, const hec_ct *b, hec_ct **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !a || !b) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_ABI_OUT1(ct_sub(c, a, b, out));
}

extern "C" hec_status ckks_drop(hec_ctx *c, const hec_ct *a, uint32_t level, hec_ct **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !a) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_ABI_OUT1(ct_drop(c, a, level, out));
}

hec_status ct_add_pt(hec_ctx *c, const hec_ct *a, const hec_pt *pt, hec_ct **out)
{
    *out = nullptr;
    if (a->level != pt->level) HEC_FAIL(HEC_ELEVEL, "level mismatch in plaintext addition");
    if (a->scale != pt->scale) HEC_FAIL(HEC_ESCALE, "scale mismatch in plaintext addition");
    const size_t nq = a->level + 1;
    u64 *t = c->alloc(nq * c->n);
    hec_ct *o = ct_clone(c, a);
    if (!t || !o) {
        c->release(t);
        ct_free(o);
        HEC_FAIL(HEC_ENOMEM, "plaintext addition buffers");
    }
    // the plaintext's Q limbs out of Montgomery form, added to c0
    hec_ew(c->T, EW_FROM_MONT, t, pt->d, nullptr, 0, 0, 0, 1, c->idmap(), (int)nq, c->st);
    hec_ew(c->T, EW_ADD, o->d, o->d, t, 0, 0, 0, 1, c->idmap(), (int)nq, c->st);
    c->release(t);
    *out = o;
    return HEC_OK;
}

extern "C" hec_status ckks_add_pt(hec_ctx *c, const hec_ct *a, const hec_pt *pt, hec_ct **out)
{
    if (!out) HEC_FAIL(HEC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c || !a || !pt) HEC_FAIL(HEC_EINVAL, "NULL argument");
    HEC_ABI_OUT1(ct_add_pt(c, a, pt, out));
}
