"""CPU oracle for RNS-CKKS -- TEST INFRASTRUCTURE ONLY.

Python front end over oracle/liboracle.so (plain C, __int128 arithmetic,
binary128 encoder).  Only tests/, the smoke check and the CPU-baseline leg of
bench.py may import this module; the product library never does.

Background (the paper's Background section, "Homomorphic encryption"):
ciphertexts are pairs over Z_Q[x]/(x^n + 1), n = 2N, with N real slots; every
multiplication consumes a level; ciphertexts support cyclic slot rotations.
The scheme conventions that the paper leaves to its library are fixed here
(and mirrored independently by the GPU library):

* primes: q_0 .. q_L then special primes p_0 .. p_{k-1}; each is the first
  prime 2^b - j*2n + 1 (j = 1, 2, ...) not already taken;
* digits of the hybrid key switch: consecutive runs of alpha = ceil((L+1)/dnum)
  primes of q_0..q_L;
* rotation by r (left: slot j <- slot j+r) is the Galois map x -> x^g with
  g = 5^(r mod N) mod 2n; rotation by 0 is the identity;
* randomness: ChaCha20 streams named (seed, purpose, index).

All ciphertexts here are in coefficient form, layout [2][level+1][n] uint64,
which is also the canonical comparison form.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        _lib = ctypes.CDLL(path)
        _declare(_lib)
    return _lib


u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)
u32p = ctypes.POINTER(ctypes.c_uint32)
dblp = ctypes.POINTER(ctypes.c_double)
MAXP = 96


class _Params(ctypes.Structure):
    _fields_ = [("logn", ctypes.c_uint32), ("n", ctypes.c_uint32), ("L", ctypes.c_uint32),
                ("k", ctypes.c_uint32), ("dnum", ctypes.c_uint32), ("alpha", ctypes.c_uint32),
                ("mod", ctypes.c_uint64 * MAXP), ("psi", ctypes.c_uint64 * MAXP)]


def _declare(L):
    P = ctypes.POINTER(_Params)
    u32, u64, dbl = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    sig = {
        "orc_mulmod": (u64, [u64, u64, u64]),
        "orc_powmod": (u64, [u64, u64, u64]),
        "orc_invmod": (u64, [u64, u64]),
        "orc_is_prime": (ctypes.c_int, [u64]),
        "orc_find_prime": (u64, [u32, u32, u64p, u32]),
        "orc_find_psi": (u64, [u64, u32]),
        "orc_params_init": (ctypes.c_int, [P, u32, u32, u32p, u32, u32p, u32]),
        "orc_ntt": (None, [u64p, u32, u64, u64]),
        "orc_intt": (None, [u64p, u32, u64, u64]),
        "orc_polymul": (None, [u64p, u64p, u64p, u32, u64, u64]),
        "orc_chacha20_block": (None, [u32p, u32, u32p, u32p]),
        "orc_stream_u64": (None, [u64, u32, u64, u64, u64, u64p]),
        "orc_sample_uniform": (None, [P, u64, u32, u64, u32p, u32, u64p]),
        "orc_sample_ternary": (None, [u64, u32, u64, u32, i64p]),
        "orc_gauss_table": (None, [dbl, u64p]),
        "orc_sample_gauss": (None, [u64, u32, u64, u32, dbl, i64p]),
        "orc_encode_direct": (ctypes.c_int, [u32, dblp, u32, dbl, i64p]),
        "orc_encode": (ctypes.c_int, [u32, dblp, u32, dbl, i64p]),
        "orc_decode": (None, [u32, dblp, dbl, dblp]),
        "orc_reduce_small": (None, [P, i64p, u32p, u32, u64p]),
        "orc_automorph": (None, [P, u32p, u32, u32, u64p, u64p]),
        "orc_keygen_secret": (None, [P, u64, i64p]),
        "orc_keygen_pk": (None, [P, u64, dbl, i64p, u64p]),
        "orc_keygen_swk": (None, [P, u64, dbl, i64p, u32, u64p]),
        "orc_keygen_swk_limbs": (None, [P, u64, dbl, i64p, u32, u32p, u32, u64p]),
        "orc_keygen_relin": (None, [P, u64, dbl, i64p, u64p]),
        "orc_encrypt": (None, [P, u64p, dbl, u64p, u32, u64, u64, u64p]),
        "orc_decrypt": (None, [P, i64p, u64p, u32, u64p]),
        "orc_modup": (None, [P, u32, u32, u64p, u64p]),
        "orc_moddown": (None, [P, u32, u64p, u64p]),
        "orc_rotate_hoisted": (None, [P, u32, u64p, u32, u32p, ctypes.POINTER(u64p), ctypes.POINTER(u64p)]),
        "orc_mul_pt": (None, [P, u32, u64p, u64p, u64p]),
        "orc_add": (None, [P, u32, u32, u64p, u64p, u64p]),
        "orc_rescale": (None, [P, u32, u64p, u64p]),
        "orc_ntt_limbs": (None, [P, u32p, u32, u64p]),
        "orc_keyswitch_raw": (None, [P, u32, u64p, u32, u32p, ctypes.POINTER(u64p), ctypes.POINTER(u64p)]),
        "orc_mul_limbs": (None, [P, u32p, u32, u64p, u64p, u64p]),
        "orc_add_limbs": (None, [P, u32p, u32, u64p, u64p, u64p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def ptr(a, t=u64p):
    return a.ctypes.data_as(t)


def u32arr(xs):
    return np.ascontiguousarray(np.asarray(xs, dtype=np.uint32))


# purposes of the random streams (must match both implementations' convention)
P_SECRET, P_PK_A, P_PK_E, P_SWK_A, P_SWK_E, P_ENC_V, P_ENC_E0, P_ENC_E1 = range(1, 9)


class Params:
    """An RNS-CKKS parameter set: ring degree n = 2^logn, ciphertext prime sizes
    qbits[0..L], special prime sizes pbits[0..k-1], dnum key-switch digits."""

    def __init__(self, logn, qbits, pbits, dnum, sigma=3.2):
        self.logn, self.n, self.N = logn, 1 << logn, 1 << (logn - 1)
        self.qbits, self.pbits = list(qbits), list(pbits)
        self.sigma = float(sigma)
        self.c = _Params()
        qb, pb = u32arr(qbits), u32arr(pbits if len(pbits) else [0])
        rc = lib().orc_params_init(ctypes.byref(self.c), logn, len(qbits), ptr(qb, u32p), len(pbits),
                                   ptr(pb, u32p), dnum)
        if rc != 0:
            raise ValueError("oracle parameter set rejected (%d)" % rc)
        self.L, self.k = self.c.L, self.c.k
        self.dnum, self.alpha = self.c.dnum, self.c.alpha
        self.mod = [int(self.c.mod[i]) for i in range(self.L + 1 + self.k)]
        self.q = self.mod[: self.L + 1]
        self.p = self.mod[self.L + 1:]
        self.psi = [int(self.c.psi[i]) for i in range(self.L + 1 + self.k)]

    @property
    def cref(self):
        return ctypes.byref(self.c)

    def galois(self, step):
        """Galois element of a left rotation by `step` slots."""
        return pow(5, step % self.N, 2 * self.n)


class Pt:
    def __init__(self, limbs, level, scale, coeffs=None):
        self.limbs, self.level, self.scale, self.coeffs = limbs, level, scale, coeffs


class Ct:
    def __init__(self, data, level, scale):
        assert data.shape[0] == 2 and data.shape[1] == level + 1
        self.data, self.level, self.scale = data, level, float(scale)

    def copy(self):
        return Ct(self.data.copy(), self.level, self.scale)


class Oracle:
    """The CPU oracle: keys, encoding, encryption and the evaluation steps."""

    def __init__(self, params, seed, key_level=None):
        """key_level: generate the rotation keys over Q_{key_level} and P only
        (the other limbs stay zero and are never read), for tests that rotate
        at low levels of a large parameter set; rotations above that level
        are refused."""
        self.p = params
        self.seed = seed
        self.key_level = key_level
        n = params.n
        self.s = np.zeros(n, dtype=np.int64)
        lib().orc_keygen_secret(params.cref, seed, ptr(self.s, i64p))
        self.pk = np.zeros((2, params.L + 1, n), dtype=np.uint64)
        lib().orc_keygen_pk(params.cref, seed, params.sigma, ptr(self.s, i64p), ptr(self.pk))
        self._swk = {}
        self._rlk = None

    # ---- keys -----------------------------------------------------------
    def swk(self, g):
        """Rotation key for Galois element g, coefficient form [dnum][2][L+1+k][n]."""
        if g not in self._swk and self.key_level is not None:
            self._swk[g] = (None, self._swk_limbs(g, self.qp_index(self.key_level)))
        if g not in self._swk:
            p = self.p
            nl = p.L + 1 + p.k
            k = np.zeros((p.dnum, 2, nl, p.n), dtype=np.uint64)
            lib().orc_keygen_swk(p.cref, self.seed, p.sigma, ptr(self.s, i64p), g, ptr(k))
            kn = k.copy()
            pidx = u32arr(list(range(nl)) * (2 * p.dnum))
            lib().orc_ntt_limbs(p.cref, ptr(pidx, u32p), 2 * p.dnum * nl, ptr(kn))
            self._swk[g] = (k, kn)
        return self._swk[g]

    def swk_limbs_coeff(self, g, pidx):
        """The rotation key of g generated on the listed primes only (coefficient
        form, full layout, other limbs zero)."""
        p = self.p
        k = np.zeros((p.dnum, 2, p.L + 1 + p.k, p.n), dtype=np.uint64)
        pl = u32arr(pidx)
        lib().orc_keygen_swk_limbs(p.cref, self.seed, p.sigma, ptr(self.s, i64p), g, ptr(pl, u32p), len(pl), ptr(k))
        return k

    def _swk_limbs(self, g, pidx):
        # NTT form of the listed limbs only (np.zeros pages never written stay unallocated)
        p = self.p
        k = self.swk_limbs_coeff(g, pidx)
        sel = np.ascontiguousarray(k[:, :, pidx, :]).reshape(-1, p.n)
        pl = u32arr(list(pidx) * (2 * p.dnum))
        lib().orc_ntt_limbs(p.cref, ptr(pl, u32p), len(pl), ptr(sel))
        k[:, :, pidx, :] = sel.reshape(p.dnum, 2, len(pidx), p.n)
        return k

    def _check_key_level(self, level):
        if self.key_level is not None and level > self.key_level:
            raise ValueError("rotation keys were generated up to level %d only" % self.key_level)

    def relin_key(self):
        """Relinearization key (s^2 target), coefficient and NTT forms [dnum][2][L+1+k][n]."""
        if self._rlk is None:
            p = self.p
            nl = p.L + 1 + p.k
            k = np.zeros((p.dnum, 2, nl, p.n), dtype=np.uint64)
            lib().orc_keygen_relin(p.cref, self.seed, p.sigma, ptr(self.s, i64p), ptr(k))
            kn = k.copy()
            pidx = u32arr(list(range(nl)) * (2 * p.dnum))
            lib().orc_ntt_limbs(p.cref, ptr(pidx, u32p), 2 * p.dnum * nl, ptr(kn))
            self._rlk = (k, kn)
        return self._rlk

    # ---- encoding ---------------------------------------------------------
    def encode_coeffs(self, z, scale):
        z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
        m = np.zeros(self.p.n, dtype=np.int64)
        rc = lib().orc_encode(self.p.n, ptr(z, dblp), len(z), float(scale), ptr(m, i64p))
        if rc != 0:
            raise OverflowError("encoded coefficient exceeds 2^62")
        return m

    def limbs_of(self, m, level):
        """Signed integer coefficients reduced mod q_0..q_level: [level+1][n]."""
        out = np.zeros((level + 1, self.p.n), dtype=np.uint64)
        pidx = u32arr(range(level + 1))
        lib().orc_reduce_small(self.p.cref, ptr(m, i64p), ptr(pidx, u32p), level + 1, ptr(out))
        return out

    def encode(self, z, level, scale):
        m = self.encode_coeffs(z, scale)
        return Pt(self.limbs_of(m, level), level, float(scale), m)

    def decode(self, m_float, scale):
        m = np.ascontiguousarray(np.asarray(m_float, dtype=np.float64))
        z = np.zeros(self.p.N, dtype=np.float64)
        lib().orc_decode(self.p.n, ptr(m, dblp), float(scale), ptr(z, dblp))
        return z

    # ---- encryption ---------------------------------------------------------
    def encrypt(self, pt, seed, index=0):
        p = self.p
        ct = np.zeros((2, pt.level + 1, p.n), dtype=np.uint64)
        lib().orc_encrypt(p.cref, ptr(self.pk), p.sigma, ptr(np.ascontiguousarray(pt.limbs)), pt.level, seed,
                          index, ptr(ct))
        return Ct(ct, pt.level, pt.scale)

    def decrypt_residues(self, ct):
        m = np.zeros((ct.level + 1, self.p.n), dtype=np.uint64)
        lib().orc_decrypt(self.p.cref, ptr(self.s, i64p), ptr(np.ascontiguousarray(ct.data)), ct.level, ptr(m))
        return m

    def crt_centered(self, res):
        """Exact centered CRT of [l+1][n] residues with Python integers."""
        qs = self.p.q[: res.shape[0]]
        Q = 1
        for q in qs:
            Q *= q
        acc = np.zeros(res.shape[1], dtype=object)
        for i, q in enumerate(qs):
            Qi = Q // q
            c = Qi * pow(Qi % q, -1, q)
            acc = acc + res[i].astype(object) * c
        acc = acc % Q
        half = Q // 2
        return np.where(acc > half, acc - Q, acc)

    def decrypt(self, ct):
        m = self.crt_centered(self.decrypt_residues(ct))
        return self.decode(np.array([float(v) for v in m]), ct.scale)

    # ---- evaluation ---------------------------------------------------------
    def rotate_hoisted(self, ct, steps):
        self._check_key_level(ct.level)
        p = self.p
        outs, gs, keys = [], [], []
        res = [None] * len(steps)
        todo = []
        for i, r in enumerate(steps):
            if r % p.N == 0:
                res[i] = ct.copy()
            else:
                todo.append(i)
        if todo:
            for i in todo:
                g = p.galois(steps[i])
                gs.append(g)
                keys.append(self.swk(g)[1])
                outs.append(np.zeros((2, ct.level + 1, p.n), dtype=np.uint64))
            kp = (u64p * len(keys))(*[ptr(k) for k in keys])
            op = (u64p * len(outs))(*[ptr(o) for o in outs])
            gsa = u32arr(gs)
            lib().orc_rotate_hoisted(p.cref, ct.level, ptr(np.ascontiguousarray(ct.data)), len(gs), ptr(gsa, u32p),
                                     kp, op)
            for i, o in zip(todo, outs):
                res[i] = Ct(o, ct.level, ct.scale)
        return res

    def rotate(self, ct, step):
        return self.rotate_hoisted(ct, [step])[0]

    def mul_pt(self, ct, pt):
        if pt.level != ct.level:
            raise ValueError("level mismatch")
        out = np.zeros_like(ct.data)
        lib().orc_mul_pt(self.p.cref, ct.level, ptr(np.ascontiguousarray(ct.data)), ptr(np.ascontiguousarray(pt.limbs)),
                         ptr(out))
        return Ct(out, ct.level, ct.scale * pt.scale)

    def add_pt(self, ct, pt):
        """ct + pt (plaintext at the ciphertext's level and scale): pt added to c0."""
        if pt.level != ct.level or pt.scale != ct.scale:
            raise ValueError("level/scale mismatch")
        qi = list(range(ct.level + 1))
        return Ct(np.stack([self.add_limbs(qi, ct.data[0], pt.limbs), ct.data[1].copy()]), ct.level, ct.scale)

    def add(self, a, b):
        if a.level != b.level or a.scale != b.scale:
            raise ValueError("level/scale mismatch")
        out = np.zeros_like(a.data)
        lib().orc_add(self.p.cref, a.level + 1, 2, ptr(np.ascontiguousarray(a.data)), ptr(np.ascontiguousarray(b.data)),
                      ptr(out))
        return Ct(out, a.level, a.scale)

    def rescale(self, ct):
        if ct.level == 0:
            raise ValueError("cannot rescale at level 0")
        out = np.zeros((2, ct.level, self.p.n), dtype=np.uint64)
        lib().orc_rescale(self.p.cref, ct.level, ptr(np.ascontiguousarray(ct.data)), ptr(out))
        return Ct(out, ct.level - 1, ct.scale / self.p.q[ct.level])

    def drop_to(self, ct, level):
        return Ct(ct.data[:, : level + 1].copy(), level, ct.scale)

    # ---- key-switch products without ModDown (lazy ModDown) ---------------
    def qp_index(self, level):
        return list(range(level + 1)) + [self.p.L + 1 + t for t in range(self.p.k)]

    def limbs_qp(self, m, level):
        """Signed integer coefficients reduced mod q_0..q_level, p_0..p_{k-1}."""
        pidx = u32arr(self.qp_index(level))
        out = np.zeros((len(pidx), self.p.n), dtype=np.uint64)
        lib().orc_reduce_small(self.p.cref, ptr(m, i64p), ptr(pidx, u32p), len(pidx), ptr(out))
        return out

    def keyswitch_raw(self, ct, steps):
        """Per step: the key-switch product (e0, e1) over Q_l and P, coefficient
        form [2][l+1+k][n], before ModDown; None for a zero rotation."""
        self._check_key_level(ct.level)
        p = self.p
        todo = [i for i, r in enumerate(steps) if r % p.N]
        res = [None] * len(steps)
        if todo:
            nqp = ct.level + 1 + p.k
            outs = [np.zeros((2, nqp, p.n), dtype=np.uint64) for _ in todo]
            gs = u32arr([p.galois(steps[i]) for i in todo])
            kp = (u64p * len(todo))(*[ptr(self.swk(int(g))[1]) for g in gs])
            op = (u64p * len(todo))(*[ptr(o) for o in outs])
            lib().orc_keyswitch_raw(p.cref, ct.level, ptr(np.ascontiguousarray(ct.data)), len(todo), ptr(gs, u32p),
                                    kp, op)
            for i, o in zip(todo, outs):
                res[i] = o
        return res

    def mul_limbs(self, pidx, a, b):
        out = np.zeros_like(a)
        pi = u32arr(pidx)
        lib().orc_mul_limbs(self.p.cref, ptr(pi, u32p), len(pi), ptr(np.ascontiguousarray(a)),
                            ptr(np.ascontiguousarray(b)), ptr(out))
        return out

    def add_limbs(self, pidx, a, b):
        out = np.zeros_like(a)
        pi = u32arr(pidx)
        lib().orc_add_limbs(self.p.cref, ptr(pi, u32p), len(pi), ptr(np.ascontiguousarray(a)),
                            ptr(np.ascontiguousarray(b)), ptr(out))
        return out

    def automorph(self, pidx, x, g):
        out = np.zeros_like(x)
        pi = u32arr(pidx)
        lib().orc_automorph(self.p.cref, ptr(pi, u32p), len(pi), g, ptr(np.ascontiguousarray(x)), ptr(out))
        return out

    def moddown(self, level, x):
        """[l+1+k][n] over Q_l and P -> [l+1][n] over Q_l (floor ModDown)."""
        out = np.zeros((level + 1, self.p.n), dtype=np.uint64)
        lib().orc_moddown(self.p.cref, level, ptr(np.ascontiguousarray(x)), ptr(out))
        return out

    # ---- ciphertext products (tensor product and relinearization) -----------
    def mul_ct(self, a, b):
        """a * b for ciphertexts at one level: (d0, d1, d2) = (a0 b0, a0 b1 + a1 b0,
        a1 b1), then d2 key-switched from s^2 to s with the relinearization key:
        (d0 + ModDown(e0), d1 + ModDown(e1)), e = sum_j ModUp_j(d2) * rlk_j.
        Scale a.scale * b.scale; not rescaled."""
        if a.level != b.level:
            raise ValueError("level mismatch")
        lvl = a.level
        qi = list(range(lvl + 1))
        d0 = self.mul_limbs(qi, a.data[0], b.data[0])
        d1 = self.add_limbs(qi, self.mul_limbs(qi, a.data[0], b.data[1]), self.mul_limbs(qi, a.data[1], b.data[0]))
        d2 = self.mul_limbs(qi, a.data[1], b.data[1])
        p = self.p
        nqp = lvl + 1 + p.k
        e = np.zeros((2, nqp, p.n), dtype=np.uint64)
        tmp = np.ascontiguousarray(np.stack([d0, d2]))   # the key switch reads the second polynomial
        gs = u32arr([1])
        kp = (u64p * 1)(ptr(self.relin_key()[1]))
        op = (u64p * 1)(ptr(e))
        lib().orc_keyswitch_raw(p.cref, lvl, ptr(tmp), 1, ptr(gs, u32p), kp, op)
        data = np.stack([self.add_limbs(qi, d0, self.moddown(lvl, e[0])),
                         self.add_limbs(qi, d1, self.moddown(lvl, e[1]))])
        return Ct(data, lvl, a.scale * b.scale)

    def const_coeffs(self, value, scale):
        """A constant in every slot encodes as the constant polynomial
        round_half_away(value * scale) (both doubles; the product taken exactly)."""
        from fractions import Fraction
        x = Fraction(float(value)) * Fraction(float(scale))
        r = int(abs(x) + Fraction(1, 2))          # floor(|x| + 1/2): half away from zero
        r = r if x >= 0 else -r
        if abs(r) >= 1 << 62:
            raise OverflowError("constant exceeds 2^62")
        m = np.zeros(self.p.n, dtype=np.int64)
        m[0] = r
        return m

    def add_const(self, ct, value, scale=None):
        """ct + value (a constant in every slot), encoded at the ciphertext's scale."""
        m = self.const_coeffs(value, ct.scale if scale is None else scale)
        pt = self.limbs_of(m, ct.level)
        qi = list(range(ct.level + 1))
        return Ct(np.stack([self.add_limbs(qi, ct.data[0], pt), ct.data[1].copy()]), ct.level, ct.scale)

    def mul_const(self, ct, value, pscale):
        """ct * value (constant in every slot) encoded at pscale; scale ct.scale * pscale."""
        m = self.const_coeffs(value, pscale)
        return self.mul_pt(ct, Pt(self.limbs_of(m, ct.level), ct.level, pscale))

    def sub(self, a, b):
        if a.level != b.level or a.scale != b.scale:
            raise ValueError("level or scale mismatch")
        qi = list(range(a.level + 1))
        return Ct(np.stack([self.add_limbs(qi, a.data[t], self.neg_limbs(qi, b.data[t])) for t in range(2)]),
                  a.level, a.scale)

    def neg_limbs(self, pidx, x):
        out = np.zeros_like(x)
        for i, l in enumerate(pidx):
            q = np.uint64(self.p.mod[l])
            nz = x[i] != 0
            out[i][nz] = q - x[i][nz]
        return out
