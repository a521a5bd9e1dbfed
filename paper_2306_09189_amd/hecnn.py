"""Thin Python binding of libhecnn.so (include/hecnn.h): argument marshalling
only -- every step of the computation runs in the HIP library.  Raises if the
library is missing; there is no fallback path."""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhecnn.so")

HEC_OK, HEC_EINVAL, HEC_ENOMEM, HEC_ELEVEL, HEC_ESCALE, HEC_ENOKEY, HEC_ELAYOUT, HEC_EDEVICE, HEC_EBUSY = range(9)
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "ELEVEL", 4: "ESCALE", 5: "ENOKEY", 6: "ELAYOUT", 7: "EDEVICE",
          8: "EBUSY"}

# every symbol the header declares
EXPORTS = [
    "hec_ctx_create", "hec_ctx_destroy", "hec_last_error", "hec_ctx_primes", "hec_ctx_slots", "ckks_keygen",
    "ckks_gen_rotation_keys", "hec_ctx_key_bytes", "hec_ctx_keyswitch_count", "ckks_encode", "ckks_encrypt", "ckks_encrypt_idx", "ckks_decrypt",
    "ckks_rotate", "ckks_rotate_hoisted", "ckks_rescale", "ckks_mul_pt", "ckks_add", "ckks_ct_info", "ckks_ct_export",
    "ckks_ct_import", "ckks_pt_export", "ckks_pt_import", "ckks_encode_coeffs", "he_image_encrypt",
    "he_image_decrypt", "he_image_info", "he_image_block_map", "he_image_shard", "he_conv2d_sharded",
    "he_conv2d_plan_create", "he_conv2d_plan_run", "he_conv2d_plan_set_mode", "he_conv2d_plan_steps",
    "he_conv2d_plan_set_downsample_mode",
    "he_avgpool_steps", "he_conv2d_plan_free", "he_avgpool", "he_avgpool_ex", "he_linear", "he_linear_steps", "hec_ct_free", "hec_pt_free", "hec_image_free",
    "hec_ctx_sync", "hec_ctx_release_cached", "hec_prof_start", "hec_prof_stop", "hec_prof_launches", "hec_probe_stream", "he_image_channel_shard",
    "ckks_sub", "ckks_mul", "ckks_mul_const", "ckks_add_const", "ckks_drop", "he_cheb_eval", "he_image_cheb_eval",
    "ckks_add_pt", "he_image_add_bias", "he_block_create", "he_block_steps", "he_block_run", "he_block_free",
    "he_conv2d_plan_create_ex", "hec_gauss_table", "ckks_rotate_noalloc",
    "hec_batch_begin", "hec_batch_add", "hec_batch_launch", "hec_batch_output", "hec_batch_size", "hec_batch_free",
    "hec_server_start", "hec_server_add_model", "hec_server_model_footprint", "hec_server_submit", "hec_server_poll",
    "hec_server_stats", "hec_server_stop",
    "hec_tune_set", "hec_tune_get", "hec_tune_describe", "hec_tune_save", "hec_tune_load", "hec_autotune_conv",
]


class HecError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class ServerParams(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_uint32), ("max_batch", ctypes.c_uint32), ("mem_budget", ctypes.c_size_t)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("batched_requests", ctypes.c_uint64), ("max_concurrent", ctypes.c_uint64),
                ("peak_mem", ctypes.c_size_t), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("req_per_s", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("L", ctypes.c_uint32), ("q0_bits", ctypes.c_uint32),
                ("q_bits", ctypes.c_uint32), ("k", ctypes.c_uint32), ("p_bits", ctypes.c_uint32),
                ("dnum", ctypes.c_uint32), ("log_scale", ctypes.c_uint32), ("sigma", ctypes.c_double),
                ("secret_dist", ctypes.c_uint32)]


_lib = None
vp = ctypes.c_void_p
u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)
i32p = ctypes.POINTER(ctypes.c_int32)
u32p = ctypes.POINTER(ctypes.c_uint32)
dblp = ctypes.POINTER(ctypes.c_double)
szp = ctypes.POINTER(ctypes.c_size_t)


def lib():
    """Load libhecnn.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhecnn.so is not built (run __graft_entry__.build()); no fallback exists")
        L = ctypes.CDLL(LIB_PATH)
        c, u32, u64, dbl, sz = ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t
        P = ctypes.POINTER
        sig = {
            "hec_ctx_create": (c, [P(Params), c, vp, P(vp)]),
            "hec_ctx_destroy": (None, [vp]),
            "hec_last_error": (ctypes.c_char_p, []),
            "hec_ctx_primes": (c, [vp, u64p, sz, szp]),
            "hec_ctx_slots": (u32, [vp]),
            "ckks_keygen": (c, [vp, u64, i32p, sz]),
            "ckks_gen_rotation_keys": (c, [vp, i32p, sz]),
            "hec_ctx_key_bytes": (sz, [vp]),
            "hec_ctx_keyswitch_count": (u64, [vp]),
            "ckks_encode": (c, [vp, dblp, sz, u32, dbl, P(vp)]),
            "ckks_encrypt": (c, [vp, vp, u64, P(vp)]),
            "ckks_encrypt_idx": (c, [vp, vp, u64, u64, P(vp)]),
            "ckks_decrypt": (c, [vp, vp, dblp, sz]),
            "ckks_rotate": (c, [vp, vp, ctypes.c_int32, P(vp)]),
            "ckks_rotate_hoisted": (c, [vp, vp, i32p, sz, P(vp)]),
            "ckks_rotate_noalloc": (c, [vp, vp, ctypes.c_int32, vp]),
            "ckks_rescale": (c, [vp, vp]),
            "ckks_mul_pt": (c, [vp, vp, vp, P(vp)]),
            "ckks_add": (c, [vp, vp, vp, P(vp)]),
            "ckks_sub": (c, [vp, vp, vp, P(vp)]),
            "ckks_mul": (c, [vp, vp, vp, P(vp)]),
            "ckks_mul_const": (c, [vp, vp, dbl, dbl, P(vp)]),
            "ckks_add_const": (c, [vp, vp, dbl, P(vp)]),
            "ckks_drop": (c, [vp, vp, u32, P(vp)]),
            "he_cheb_eval": (c, [vp, vp, dblp, sz, dbl, dbl, P(vp)]),
            "he_image_cheb_eval": (c, [vp, vp, dblp, sz, dbl, dbl, P(vp)]),
            "ckks_add_pt": (c, [vp, vp, vp, P(vp)]),
            "he_image_add_bias": (c, [vp, vp, dblp, P(vp)]),
            "he_block_create": (c, [vp, vp, dblp, u32, dblp, dblp, u32, dblp, u32, dbl, dblp, sz, c, P(vp)]),
            "he_block_steps": (c, [vp, i32p, sz, szp]),
            "he_block_run": (c, [vp, vp, vp, P(vp)]),
            "he_block_free": (None, [vp]),
            "ckks_ct_info": (c, [vp, u32p, dblp]),
            "ckks_ct_export": (c, [vp, vp, u64p, u32p, dblp]),
            "ckks_ct_import": (c, [vp, u64p, u32, dbl, P(vp)]),
            "ckks_pt_export": (c, [vp, vp, u64p, u32p, dblp]),
            "ckks_pt_import": (c, [vp, u64p, u32, dbl, P(vp)]),
            "ckks_encode_coeffs": (c, [vp, dblp, sz, dbl, i64p]),
            "he_image_encrypt": (c, [vp, dblp, u32, u32, u32, u32, u64, P(vp)]),
            "he_image_decrypt": (c, [vp, vp, dblp]),
            "he_image_info": (c, [vp, u32p, u32p, u32p, u32p, u32p]),
            "he_image_block_map": (c, [vp, u32, i32p, sz]),
            "he_image_shard": (vp, [vp, u32]),
            "he_conv2d_sharded": (c, [vp, vp, dblp, u32, u32, u32, u32, u32, dblp, P(vp)]),
            "he_conv2d_plan_create": (c, [vp, vp, dblp, u32, u32, u32, u32, u32, P(vp)]),
            "he_conv2d_plan_run": (c, [vp, vp, vp, P(vp)]),
            "he_conv2d_plan_create_ex": (c, [vp, vp, dblp, u32, u32, u32, u32, u32, u32, P(vp)]),
            "he_conv2d_plan_set_mode": (c, [vp, c]),
            "he_conv2d_plan_set_downsample_mode": (c, [vp, c]),
            "he_conv2d_plan_steps": (c, [vp, i32p, sz, szp]),
            "he_avgpool_steps": (c, [vp, vp, i32p, sz, szp]),
            "he_linear_steps": (c, [vp, vp, i32p, sz, szp]),
            "he_linear": (c, [vp, vp, dblp, u32, c, P(vp)]),
            "he_conv2d_plan_free": (None, [vp]),
            "he_avgpool": (c, [vp, vp, u32, P(vp)]),
            "he_avgpool_ex": (c, [vp, vp, u32, c, P(vp)]),
            "hec_ct_free": (None, [vp]),
            "hec_pt_free": (None, [vp]),
            "hec_image_free": (None, [vp]),
            "hec_ctx_sync": (c, [vp]),
            "hec_ctx_release_cached": (c, [vp]),
            "hec_prof_start": (c, [vp, ctypes.c_char_p]),
            "hec_prof_stop": (c, [vp, u64p, u64p, dblp]),
            "hec_prof_launches": (u64, [ctypes.c_char_p]),
            "hec_probe_stream": (c, [vp, ctypes.c_int, ctypes.c_int, u64, ctypes.c_int, dblp]),
            "he_image_channel_shard": (c, [vp, u32, i32p, i32p]),
            "hec_gauss_table": (c, [dbl, u64p, sz]),
            "hec_batch_begin": (c, [vp, P(vp)]),
            "hec_batch_add": (c, [vp, vp, vp, u32p]),
            "hec_batch_launch": (c, [vp, c]),
            "hec_batch_output": (vp, [vp, u32]),
            "hec_batch_size": (u32, [vp]),
            "hec_batch_free": (None, [vp]),
            "hec_server_start": (c, [vp, P(ServerParams), P(vp)]),
            "hec_server_add_model": (c, [vp, vp, c, vp, u32p]),
            "hec_server_model_footprint": (sz, [vp, u32]),
            "hec_server_submit": (c, [vp, u32, vp, P(ctypes.c_uint64)]),
            "hec_server_poll": (c, [vp, ctypes.c_uint64, c, P(vp), dblp]),
            "hec_server_stats": (c, [vp, P(ServerStats)]),
            "hec_server_stop": (c, [vp]),
            "hec_tune_set": (c, [ctypes.c_char_p, ctypes.c_int64]),
            "hec_tune_get": (c, [ctypes.c_char_p, i64p]),
            "hec_tune_describe": (c, [ctypes.c_char_p, sz]),
            "hec_tune_save": (c, [ctypes.c_char_p]),
            "hec_tune_load": (c, [ctypes.c_char_p]),
            "hec_autotune_conv": (c, [vp, vp, vp, u32, ctypes.c_char_p, sz]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def gauss_table(sigma):
    """The 19 thresholds of the library's discrete Gaussian sampler (host only)."""
    T = np.zeros(19, dtype=np.uint64)
    check(lib().hec_gauss_table(float(sigma), _p(T, u64p), len(T)))
    return T


def tune_set(name, value):
    check(lib().hec_tune_set(name.encode(), int(value)))


def tune_get(name):
    v = ctypes.c_int64()
    check(lib().hec_tune_get(name.encode(), ctypes.byref(v)))
    return v.value


def tune_describe():
    buf = ctypes.create_string_buffer(512)
    check(lib().hec_tune_describe(buf, len(buf)))
    return buf.value.decode()


def tune_save(path):
    check(lib().hec_tune_save(os.fsencode(path)))


def tune_load(path):
    check(lib().hec_tune_load(os.fsencode(path)))


def check(status):
    if status != HEC_OK:
        raise HecError(status, lib().hec_last_error().decode())


def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _p(a, t):
    return a.ctypes.data_as(t)


class _Handle:
    """A native handle that belongs to a context.  The context's native
    destruction waits until every handle of it is freed: objects collected
    together as cyclic garbage (for instance a script's globals at interpreter
    exit) are finalized in no particular order, and a handle freed after its
    context would touch freed memory."""
    _free_fn = None

    def __init__(self, ctx, handle, owned=True):
        self.ctx, self.h, self._owned = ctx, handle, bool(owned and handle)
        if self._owned:
            ctx._retain()

    def free(self):
        if self.h:
            h, self.h = self.h, None
            if self._owned:
                self._owned = False
                try:
                    getattr(lib(), self._free_fn)(h)
                finally:
                    self.ctx._release()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Ciphertext(_Handle):
    _free_fn = "hec_ct_free"

    def info(self):
        lvl, sc = ctypes.c_uint32(), ctypes.c_double()
        check(lib().ckks_ct_info(self.h, ctypes.byref(lvl), ctypes.byref(sc)))
        return lvl.value, sc.value

    @property
    def level(self):
        return self.info()[0]

    @property
    def scale(self):
        return self.info()[1]

    def export(self):
        """Canonical form: [2][level+1][n] uint64, coefficient domain."""
        lvl = self.level
        out = np.zeros((2, lvl + 1, self.ctx.n), dtype=np.uint64)
        check(lib().ckks_ct_export(self.ctx.h, self.h, _p(out, u64p), None, None))
        return out


class Plaintext(_Handle):
    _free_fn = "hec_pt_free"

    def __init__(self, ctx, handle, level, scale):
        super().__init__(ctx, handle)
        self.level, self.scale = level, scale

    def export(self):
        out = np.zeros((self.level + 1, self.ctx.n), dtype=np.uint64)
        check(lib().ckks_pt_export(self.ctx.h, self.h, _p(out, u64p), None, None))
        return out


class Image(_Handle):
    _free_fn = "hec_image_free"

    def info(self):
        v = [ctypes.c_uint32() for _ in range(5)]
        check(lib().he_image_info(self.h, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)  # C, H, W, mp, n_shards

    def channel_shard(self, u):
        """(channel, part) of shard u of a channel-sharded image."""
        f, p = ctypes.c_int32(), ctypes.c_int32()
        check(lib().he_image_channel_shard(self.h, u, ctypes.byref(f), ctypes.byref(p)))
        return f.value, p.value

    def is_channel_sharded(self):
        C, H, W, mp, t = self.info()
        return mp * mp > self.ctx.N

    def block_map(self, u):
        C, H, W, mp, t = self.info()
        lam = np.zeros(self.ctx.N // (mp * mp), dtype=np.int32)
        check(lib().he_image_block_map(self.h, u, _p(lam, i32p), len(lam)))
        return lam

    def shard_export(self, u):
        h = lib().he_image_shard(self.h, u)
        if not h:
            raise IndexError(u)
        return Ciphertext(self.ctx, h, owned=False).export()

    def shard_info(self, u):
        h = lib().he_image_shard(self.h, u)
        lvl, sc = ctypes.c_uint32(), ctypes.c_double()
        check(lib().ckks_ct_info(h, ctypes.byref(lvl), ctypes.byref(sc)))
        return lvl.value, sc.value

    def shard_decrypt(self, u):
        """The N slot values of shard u (client side: decrypt and decode)."""
        h = lib().he_image_shard(self.h, u)
        if not h:
            raise IndexError(u)
        z = np.zeros(self.ctx.N)
        check(lib().ckks_decrypt(self.ctx.h, h, _p(z, dblp), len(z)))
        return z

    def decrypt(self):
        C, H, W, mp, t = self.info()
        x = np.zeros((C, H, W))
        check(lib().he_image_decrypt(self.ctx.h, self.h, _p(x, dblp)))
        return x


class Block(_Handle):
    _free_fn = "he_block_free"

    def steps(self):
        n = ctypes.c_size_t()
        check(lib().he_block_steps(self.h, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=np.int32)
        check(lib().he_block_steps(self.h, _p(out, i32p), len(out), ctypes.byref(n)))
        return [int(x) for x in out]

    def run(self, img):
        out = vp()
        check(lib().he_block_run(self.ctx.h, self.h, img.h, ctypes.byref(out)))
        return Image(self.ctx, out.value)


class ConvPlan(_Handle):
    _free_fn = "he_conv2d_plan_free"

    def steps(self):
        n = ctypes.c_size_t()
        check(lib().he_conv2d_plan_steps(self.h, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=np.int32)
        check(lib().he_conv2d_plan_steps(self.h, _p(out, i32p), len(out), ctypes.byref(n)))
        return [int(x) for x in out]

    def set_mode(self, mode):
        check(lib().he_conv2d_plan_set_mode(self.h, int(mode)))

    def set_downsample_mode(self, mode):
        """Form of a stride-2 plan's downsampling: -1 (the plan mode's own), 0, 2 or 4."""
        check(lib().he_conv2d_plan_set_downsample_mode(self.h, int(mode)))

    def run(self, img):
        out = vp()
        check(lib().he_conv2d_plan_run(self.ctx.h, self.h, img.h, ctypes.byref(out)))
        return Image(self.ctx, out.value)


HEC_BATCH_EAGER, HEC_BATCH_GRAPH = 0, 1


class Batch(_Handle):
    """(plan, image) items run as one launch: eagerly, or recorded once into a
    HIP graph and replayed (graph=True).  Keeps its items' plans and images."""
    _free_fn = "hec_batch_free"

    def __init__(self, ctx, handle):
        super().__init__(ctx, handle)
        self._keep = []

    def add(self, plan, img):
        i = ctypes.c_uint32()
        check(lib().hec_batch_add(self.h, plan.h, img.h, ctypes.byref(i)))
        self._keep.append((plan, img))
        return i.value

    def launch(self, graph=False):
        check(lib().hec_batch_launch(self.h, HEC_BATCH_GRAPH if graph else HEC_BATCH_EAGER))

    def __len__(self):
        return lib().hec_batch_size(self.h)

    def output(self, i):
        """Borrowed output image of item i from the last launch (valid while the batch lives
        and, for eager launches, until the next eager launch)."""
        h = lib().hec_batch_output(self.h, int(i))
        if not h:
            raise IndexError(i)
        img = Image(self.ctx, h, owned=False)
        img._batch = self
        return img


class Server:
    """Request loop over a context (lanes, memory admission, continuous
    batching); see hec_server_* in include/hecnn.h.  Keeps submitted images
    alive until their results are polled; results it hands out are freed by
    stop() (they live in the server's memory)."""

    def __init__(self, ctx, lanes=2, max_batch=4, mem_budget=32 << 30):
        self.ctx = ctx
        prm = ServerParams(int(lanes), int(max_batch), int(mem_budget))
        h = vp()
        check(lib().hec_server_start(ctx.h, ctypes.byref(prm), ctypes.byref(h)))
        self.h = h.value
        self._keep, self._inputs, self._results = [], {}, []

    def add_model(self, plan, like, pool_mode=-1):
        m = ctypes.c_uint32()
        check(lib().hec_server_add_model(self.h, plan.h, int(pool_mode), like.h, ctypes.byref(m)))
        self._keep.append((plan, like))
        return m.value

    def footprint(self, model):
        return lib().hec_server_model_footprint(self.h, int(model))

    def submit(self, model, img):
        rid = ctypes.c_uint64()
        check(lib().hec_server_submit(self.h, int(model), img.h, ctypes.byref(rid)))
        self._inputs[rid.value] = img
        return rid.value

    def poll(self, rid, wait=True):
        """-> (Image, latency_ms) when done, None when not (wait=False); raises HecError if it failed."""
        out, lat = vp(), ctypes.c_double()
        st = lib().hec_server_poll(self.h, int(rid), int(bool(wait)), ctypes.byref(out), ctypes.byref(lat))
        if st == HEC_EBUSY and not wait:
            return None
        self._inputs.pop(rid, None)
        check(st)
        img = Image(self.ctx, out.value)
        self._results.append(img)
        return img, lat.value

    def stats(self):
        st = ServerStats()
        check(lib().hec_server_stats(self.h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def stop(self):
        if self.h:
            for img in self._results:
                img.free()
            self._results = []
            h, self.h = self.h, None
            check(lib().hec_server_stop(h))
            self._inputs.clear()


class Context:
    """An RNS-CKKS context on one HIP device; `stream` is a hipStream_t (int or
    None), e.g. torch.cuda.current_stream().cuda_stream."""

    def __init__(self, log_n, L, q0_bits, q_bits, k, p_bits, dnum, log_scale, sigma=3.2, device=0, stream=None):
        self.prm = Params(log_n, L, q0_bits, q_bits, k, p_bits, dnum, log_scale, sigma, 0)
        h = vp()
        check(lib().hec_ctx_create(ctypes.byref(self.prm), device, stream, ctypes.byref(h)))
        self.h = h.value
        self.n = 1 << log_n
        self.N = self.n // 2
        self.L, self.k = L, k
        self._live, self._close_pending = 0, False

    def _retain(self):
        self._live += 1

    def _release(self):
        self._live -= 1
        if self._live == 0 and self._close_pending:
            self._destroy()

    def _destroy(self):
        h, self.h = self.h, None
        self._close_pending = False
        if h:
            lib().hec_ctx_destroy(h)

    def close(self):
        """Destroy the native context, or, while handles of it are alive, when
        the last of them is freed."""
        if getattr(self, "h", None):
            if getattr(self, "_live", 0) > 0:
                self._close_pending = True
            else:
                self._destroy()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def primes(self):
        n = ctypes.c_size_t()
        check(lib().hec_ctx_primes(self.h, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=np.uint64)
        check(lib().hec_ctx_primes(self.h, _p(out, u64p), len(out), ctypes.byref(n)))
        return [int(x) for x in out]

    def keygen(self, seed, steps=()):
        st = _arr(list(steps) or [0], np.int32)
        check(lib().ckks_keygen(self.h, seed, _p(st, i32p), len(steps)))

    def gen_rotation_keys(self, steps):
        st = _arr(list(steps) or [0], np.int32)
        check(lib().ckks_gen_rotation_keys(self.h, _p(st, i32p), len(steps)))

    def key_bytes(self):
        return lib().hec_ctx_key_bytes(self.h)

    def keyswitch_count(self):
        return int(lib().hec_ctx_keyswitch_count(self.h))

    def encode(self, z, level, scale):
        z = _arr(z, np.float64)
        out = vp()
        check(lib().ckks_encode(self.h, _p(z, dblp), len(z), level, float(scale), ctypes.byref(out)))
        return Plaintext(self, out.value, level, float(scale))

    def encode_coeffs(self, z, scale):
        z = _arr(z, np.float64)
        m = np.zeros(self.n, dtype=np.int64)
        check(lib().ckks_encode_coeffs(self.h, _p(z, dblp), len(z), float(scale), _p(m, i64p)))
        return m

    def pt_import(self, coeff, level, scale):
        coeff = _arr(coeff, np.uint64)
        out = vp()
        check(lib().ckks_pt_import(self.h, _p(coeff, u64p), level, float(scale), ctypes.byref(out)))
        return Plaintext(self, out.value, level, float(scale))

    def encrypt(self, pt, seed, index=0):
        out = vp()
        check(lib().ckks_encrypt_idx(self.h, pt.h, seed, index, ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def decrypt(self, ct, nz=None):
        nz = self.N if nz is None else nz
        z = np.zeros(nz)
        check(lib().ckks_decrypt(self.h, ct.h, _p(z, dblp), nz))
        return z

    def ct_import(self, coeff, level, scale):
        coeff = _arr(coeff, np.uint64)
        out = vp()
        check(lib().ckks_ct_import(self.h, _p(coeff, u64p), level, float(scale), ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def rotate(self, ct, step):
        out = vp()
        check(lib().ckks_rotate(self.h, ct.h, int(step), ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def rotate_noalloc(self, ct, step, out):
        """ct rotated by step into the existing ciphertext out (same level):
        the allocation-free entry point; returns out."""
        check(lib().ckks_rotate_noalloc(self.h, ct.h, int(step), out.h))
        return out

    def rotate_hoisted(self, ct, steps):
        st = _arr(steps, np.int32)
        outs = (vp * len(st))()
        check(lib().ckks_rotate_hoisted(self.h, ct.h, _p(st, i32p), len(st), outs))
        return [Ciphertext(self, o) for o in outs]

    def rescale(self, ct):
        check(lib().ckks_rescale(self.h, ct.h))
        return ct

    def mul_pt(self, ct, pt):
        out = vp()
        check(lib().ckks_mul_pt(self.h, ct.h, pt.h, ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def add(self, a, b):
        out = vp()
        check(lib().ckks_add(self.h, a.h, b.h, ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def sub(self, a, b):
        out = vp()
        check(lib().ckks_sub(self.h, a.h, b.h, ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def mul(self, a, b):
        """Ciphertext product with relinearization (not rescaled)."""
        out = vp()
        check(lib().ckks_mul(self.h, a.h, b.h, ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def mul_const(self, ct, value, pscale):
        out = vp()
        check(lib().ckks_mul_const(self.h, ct.h, float(value), float(pscale), ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def add_const(self, ct, value):
        out = vp()
        check(lib().ckks_add_const(self.h, ct.h, float(value), ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def drop(self, ct, level):
        out = vp()
        check(lib().ckks_drop(self.h, ct.h, int(level), ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def cheb_eval(self, x, coeffs, a, b):
        """sum_k coeffs[k] T_k((2x - a - b)/(b - a)) on a ciphertext or, slotwise, on every shard of an image."""
        cf = _arr(coeffs, np.float64)
        out = vp()
        if isinstance(x, Image):
            check(lib().he_image_cheb_eval(self.h, x.h, _p(cf, dblp), len(cf), float(a), float(b),
                                           ctypes.byref(out)))
            return Image(self, out.value)
        check(lib().he_cheb_eval(self.h, x.h, _p(cf, dblp), len(cf), float(a), float(b), ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def add_pt(self, ct, pt):
        out = vp()
        check(lib().ckks_add_pt(self.h, ct.h, pt.h, ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def add_bias(self, img, bias):
        """Per-channel bias on every valid pixel of each channel."""
        b = _arr(bias, np.float64)
        out = vp()
        check(lib().he_image_add_bias(self.h, img.h, _p(b, dblp), ctypes.byref(out)))
        return Image(self, out.value)

    def block(self, like, w1, bn1, w2, bn2, bound, coeffs, mode=0):
        """Basic block: conv(w1, bn1 folded) -> activation series on [-1, 1] -> conv(w2, bn2) -> 2x2 avg pool.
        bn = (gamma, shift) per output channel; bn2 may be None."""
        w1, w2 = _arr(w1, np.float64), _arr(w2, np.float64)
        C1, C2, k = w1.shape[0], w2.shape[0], w1.shape[2]
        b1 = _arr(np.concatenate([np.asarray(bn1[0], np.float64), np.asarray(bn1[1], np.float64)]), np.float64)
        b2 = None if bn2 is None else _arr(np.concatenate([np.asarray(bn2[0], np.float64),
                                                           np.asarray(bn2[1], np.float64)]), np.float64)
        cf = _arr(coeffs, np.float64)
        out = vp()
        check(lib().he_block_create(self.h, like.h, _p(w1, dblp), C1, _p(b1, dblp), _p(w2, dblp), C2,
                                    None if b2 is None else _p(b2, dblp), k, float(bound), _p(cf, dblp), len(cf),
                                    int(mode), ctypes.byref(out)))
        return Block(self, out.value)

    def image_encrypt(self, x, level, seed):
        x = _arr(x, np.float64)
        C, H, W = x.shape
        out = vp()
        check(lib().he_image_encrypt(self.h, _p(x, dblp), C, H, W, level, seed, ctypes.byref(out)))
        return Image(self, out.value)

    @staticmethod
    def _conv_weights(img, w):
        w = _arr(w, np.float64)
        if w.ndim != 4:
            raise ValueError("weights must be [Co][Ci][kh][kw]")
        if w.shape[1] != img.info()[0]:
            raise ValueError("weights have %d input channels, the image %d" % (w.shape[1], img.info()[0]))
        return w

    def conv2d(self, img, w, stride=1, pad=1, bias=None):
        """bias: Co per-channel shifts (a folded batch norm) added to the output, or None."""
        w = self._conv_weights(img, w)
        Co, Ci, kh, kw = w.shape
        b = None
        if bias is not None:
            b = _arr(bias, np.float64)
            if b.shape != (Co,):
                raise ValueError("bias must hold Co = %d values" % Co)
        out = vp()
        check(lib().he_conv2d_sharded(self.h, img.h, _p(w, dblp), Co, kh, kw, stride, pad,
                                      None if b is None else _p(b, dblp), ctypes.byref(out)))
        return Image(self, out.value)

    def conv2d_plan(self, like, w, stride=1, pad=1, q_only=False, basis=None):
        """q_only: weight plaintexts over Q only (modes 0 and 1), for layers too large otherwise.
        basis = s: weight plaintexts in basis-mask form, tap masks per block encoded at 2^s (modes 0-2)."""
        w = self._conv_weights(like, w)
        Co, Ci, kh, kw = w.shape
        out = vp()
        flags = (1 if q_only else 0) | ((2 | (int(basis) << 8)) if basis is not None else 0)
        if flags:
            check(lib().he_conv2d_plan_create_ex(self.h, like.h, _p(w, dblp), Co, kh, kw, stride, pad, flags,
                                                 ctypes.byref(out)))
        else:
            check(lib().he_conv2d_plan_create(self.h, like.h, _p(w, dblp), Co, kh, kw, stride, pad,
                                              ctypes.byref(out)))
        return ConvPlan(self, out.value)

    def avgpool(self, img, mode=0):
        out = vp()
        if mode == 0:
            check(lib().he_avgpool(self.h, img.h, 2, ctypes.byref(out)))
        else:
            check(lib().he_avgpool_ex(self.h, img.h, 2, int(mode), ctypes.byref(out)))
        return Image(self, out.value)

    def avgpool_steps(self, img):
        n = ctypes.c_size_t()
        check(lib().he_avgpool_steps(self.h, img.h, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=np.int32)
        check(lib().he_avgpool_steps(self.h, img.h, _p(out, i32p), len(out), ctypes.byref(n)))
        return [int(x) for x in out]

    def linear(self, img, W, pool=False):
        """Linear (W [O][C*H*W]) or pool-linear (W [O][C]) layer: one ciphertext, output o in slot o."""
        W = np.ascontiguousarray(W, dtype=np.float64)
        out = vp()
        check(lib().he_linear(self.h, img.h, _p(W, dblp), W.shape[0], int(bool(pool)), ctypes.byref(out)))
        return Ciphertext(self, out.value)

    def linear_steps(self, img):
        n = ctypes.c_size_t()
        check(lib().he_linear_steps(self.h, img.h, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=np.int32)
        check(lib().he_linear_steps(self.h, img.h, _p(out, i32p), len(out), ctypes.byref(n)))
        return [int(x) for x in out]

    def autotune_conv(self, plan, img, reps=3):
        """Pick the launch parameters for plan.run(img) (bit-identical output); returns the report."""
        buf = ctypes.create_string_buffer(4096)
        check(lib().hec_autotune_conv(self.h, plan.h, img.h, int(reps), buf, len(buf)))
        return buf.value.decode()

    def batch(self):
        out = vp()
        check(lib().hec_batch_begin(self.h, ctypes.byref(out)))
        return Batch(self, out.value)

    def sync(self):
        check(lib().hec_ctx_sync(self.h))

    def release_cached(self):
        """Device memory cached by the library's pools back to the device."""
        check(lib().hec_ctx_release_cached(self.h))

    def prof_start(self, kernel):
        check(lib().hec_prof_start(self.h, kernel.encode()))

    def prof_stop(self):
        """-> (launches, units, total_ms) of the kernel selected by prof_start."""
        a, b, t = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_double()
        check(lib().hec_prof_stop(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(t)))
        return a.value, b.value, t.value

    def probe_stream(self, nread, nwrite, words, reps=20):
        """Average microseconds per launch of a kernel that reads `nread` and
        writes `nwrite` streams of `words` 64-bit words (no arithmetic)."""
        t = ctypes.c_double()
        check(lib().hec_probe_stream(self.h, nread, nwrite, words, reps, ctypes.byref(t)))
        return t.value

    @staticmethod
    def prof_launches(kernel):
        """Launches of `kernel` since the library was loaded."""
        return lib().hec_prof_launches(kernel.encode())
