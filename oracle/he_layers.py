"""Homomorphic convolution and 2x2 average pooling -- oracle side (TEST ONLY).

The schedule of the paper's Section 4 ("Homomorphic Neural Network
Operators"), written once over an abstract backend so that it can run either
on encrypted oracle ciphertexts (`CkksBackend`) or on cleartext FP64 slot
vectors (`SlotSim`, where a rotation is `np.roll` and a plaintext product is an
elementwise product).  The slot simulator checks the layout algebra against a
direct FP64 convolution; the encrypted backend gives the bit-exact ciphertexts
the GPU library must reproduce.

Layout (Section 4, "Sharding and Encrypting an Image", "Duplicating and
Permuting Channels"): every channel is stored row-major in a block of
B = mp*mp slots, mp the channel side padded to a power of two (dimensions that
are not powers of two are zero padded, as the paper allows); a shard holds
N/B blocks.  Each shard carries a block map lam[b] = logical channel held by
block b (-1 for an empty block); duplication and the permutation introduced by
pooling are both just block maps.

Readings of passages that are silent, garbled or ambiguous:
  * duplicated channels are stored as consecutive copies, [M0, M0, M1, M1, ...],
    the order the pooling duplication step produces;
  * the offsets of a convolution are found by the two-phase rule in
    `_rotation_offsets` (offsets that serve every output block first, then any
    block still missing a channel), smallest offset first;
  * horizontal reduction keeps column 2i (even rows only) and shifts it left by
    i; vertical reduction takes the left half of row 2j and shifts it left by
    3j*mp/2 (the printed equation's "3i" read as 3j);
  * the 1/4 of the average is folded into the horizontal masks;
  * consolidation shifts shard e of a group right by e*B/4 (the printed
    equation repeats S_2 and writes m^2 for the post-pool block size);
    duplication by d shifts by multiples of B/d;
  * when only one level is left, the two reductions are fused into one
    masked sum (masks combined non-homomorphically) with masks at scale q/4;
  * a convolution's weight plaintexts may be built in basis-mask form: the
    plaintext of a tap is, block by block, a weight times the tap's mask, so
    it is sum_b round(w_b q_l / 2^s) * E_b with E_b the encoding of the mask
    restricted to block b at scale 2^s (an exact integer combination of a few
    basis polynomials instead of one encoding per weight plaintext).
"""
import math

import numpy as np


def next_pow2(x):
    return 1 << max(0, (int(x) - 1).bit_length())


class Layout:
    """Where each channel of a C x H x W image lives in a list of shards."""

    def __init__(self, N, C, H, W, mp, kind, shards):
        self.N, self.C, self.H, self.W, self.mp = N, C, H, W, mp
        self.B = mp * mp
        self.kind = kind          # "image" or "channel"
        self.shards = shards      # image: list of block maps; channel: list of (channel, part)

    @property
    def nb(self):
        return self.N // self.B

    def copy(self):
        return Layout(self.N, self.C, self.H, self.W, self.mp, self.kind, [list(s) if isinstance(s, list) else s
                                                                           for s in self.shards])

    def __repr__(self):
        return "Layout(%s C=%d %dx%d mp=%d shards=%d)" % (self.kind, self.C, self.H, self.W, self.mp,
                                                          len(self.shards))


def natural_layout(N, C, H, W, mp=None):
    """Channel-major row-major packing; channels spread over image shards when
    m^2 c > N; a channel split into consecutive-row channel shards when
    m^2 > N; d = N/(m^2 c) consecutive copies when the image underfills a shard
    (Section 4, sharding and duplication paragraphs)."""
    if mp is None:
        mp = next_pow2(max(H, W))
    B = mp * mp
    if B <= N:
        nb = N // B
        Cp = next_pow2(C)
        if Cp * B <= N:
            d = N // (Cp * B)
            return Layout(N, C, H, W, mp, "image", [[b // d if b // d < C else -1 for b in range(nb)]])
        t = -(-C // nb)   # no shard is left entirely empty
        return Layout(N, C, H, W, mp, "image",
                      [[u * nb + b if u * nb + b < C else -1 for b in range(nb)] for u in range(t)])
    spc = B // N
    return Layout(N, C, H, W, mp, "channel", [(f, part) for f in range(C) for part in range(spc)])


def pack(x, lay):
    """Cleartext image [C][H][W] -> list of slot vectors (one per shard)."""
    N, mp, B = lay.N, lay.mp, lay.B
    out = []
    for s in lay.shards:
        v = np.zeros(N)
        if lay.kind == "image":
            for b, f in enumerate(s):
                if f >= 0:
                    blk = np.zeros((mp, mp))
                    blk[: lay.H, : lay.W] = x[f]
                    v[b * B:(b + 1) * B] = blk.reshape(-1)
        else:
            f, part = s
            R = N // mp
            blk = np.zeros((mp, mp))
            blk[: lay.H, : lay.W] = x[f]
            v[:] = blk[part * R:(part + 1) * R].reshape(-1)
        out.append(v)
    return out


def unpack(vecs, lay):
    """Slot vectors -> image [C][H][W], reading the first copy of each channel."""
    mp, B = lay.mp, lay.B
    x = np.full((lay.C, lay.H, lay.W), np.nan)
    if lay.kind == "image":
        seen = set()
        for u, s in enumerate(lay.shards):
            for b, f in enumerate(s):
                if f >= 0 and f not in seen:
                    seen.add(f)
                    x[f] = np.asarray(vecs[u][b * B:(b + 1) * B]).reshape(mp, mp)[: lay.H, : lay.W]
    else:
        R = lay.N // mp
        full = np.zeros((lay.C, mp, mp))
        for u, (f, part) in enumerate(lay.shards):
            full[f, part * R:(part + 1) * R] = np.asarray(vecs[u]).reshape(R, mp)
        x = full[:, : lay.H, : lay.W]
    return x


# ---------------------------------------------------------------------------
# backends
# ---------------------------------------------------------------------------

class SlotSim:
    """Cleartext slot vectors: rotation is np.roll, products are elementwise.
    A value is (vector, level, scale) with level/scale bookkeeping only."""

    def __init__(self, N, qs):
        self.N, self.qs = N, qs

    def q(self, level):
        return float(self.qs[level])

    def rotate_hoisted(self, ct, steps):
        v, lvl, sc = ct
        return [(np.roll(v, -(r % self.N)), lvl, sc) for r in steps]

    def rotate(self, ct, r):
        return self.rotate_hoisted(ct, [r])[0]

    def mul_plain(self, ct, vec, pscale):
        v, lvl, sc = ct
        return (v * vec, lvl, sc * pscale)

    def add(self, a, b):
        assert a[1] == b[1]
        return (a[0] + b[0], a[1], a[2])

    def add_plain(self, ct, vec):
        v, lvl, sc = ct
        return (v + vec, lvl, sc)

    def rescale(self, ct):
        v, lvl, sc = ct
        assert lvl > 0
        return (v, lvl - 1, sc / self.qs[lvl])

    def level(self, ct):
        return ct[1]


class BlockVec(np.ndarray):
    """A slot vector that is, block by block, a weight times one common 0/1
    mask of B slots: vec[b*B:(b+1)*B] = wb[b] * mask (the weight plaintext of
    one convolution tap, Section 4.1).  Arrays derived from it (rolls,
    products, slices) are plain vectors again."""

    def __new__(cls, N, B, mask):
        obj = np.zeros(N).view(cls)
        obj.B, obj.mask, obj.wb = B, mask, {}
        return obj

    def __array_finalize__(self, obj):
        self.B, self.mask, self.wb = None, None, {}

    def set_block(self, b, w):
        self[b * self.B:(b + 1) * self.B] = w * self.mask
        self.wb[b] = float(w)


class CkksBackend:
    """Encrypted oracle ciphertexts; a plaintext product encodes the slot
    vector at the requested scale, at the ciphertext's level.  With basis = s
    the block-masked weight vectors of a convolution are built in basis-mask
    form instead (`pt_coeffs`)."""

    def __init__(self, oracle, basis=None):
        self.o = oracle
        self.basis = basis
        self._E = {}

    def _basis_poly(self, vec, b):
        """E_b: the encoding of vec's mask restricted to block b at scale 2^s."""
        key = (vec.mask.tobytes(), vec.B, b)
        if key not in self._E:
            z = np.zeros(len(vec))
            z[b * vec.B:(b + 1) * vec.B] = vec.mask
            self._E[key] = self.o.encode_coeffs(z, 2.0 ** self.basis)
        return self._E[key]

    def pt_coeffs(self, vec, pscale):
        """Integer coefficients of the plaintext of vec at pscale.  Exact
        encoding, or for a block-masked vector with basis = s:
        sum over its blocks of round_half_away(w_b * pscale / 2^s) * E_b,
        every weight rounded as a constant (exact product) and the sum taken
        over the integers."""
        if self.basis is None or getattr(vec, "mask", None) is None:
            return self.o.encode_coeffs(vec, pscale)
        wscale = float(pscale) / 2.0 ** self.basis
        m = np.zeros(self.o.p.n, dtype=np.int64)
        bound = 0
        for b, w in sorted(vec.wb.items()):
            wh = int(self.o.const_coeffs(w, wscale)[0])
            if wh == 0:
                continue
            E = self._basis_poly(vec, b)
            bound += abs(wh) * int(np.abs(E).max())
            if bound >= 1 << 62:
                raise OverflowError("basis plaintext coefficient exceeds 2^62")
            m += wh * E
        return m

    def q(self, level):
        return float(self.o.p.q[level])

    def rotate_hoisted(self, ct, steps):
        return self.o.rotate_hoisted(ct, steps)

    def rotate(self, ct, r):
        return self.o.rotate(ct, r)

    def mul_plain(self, ct, vec, pscale):
        from .ckks import Pt
        m = self.pt_coeffs(vec, pscale)
        return self.o.mul_pt(ct, Pt(self.o.limbs_of(m, ct.level), ct.level, float(pscale), m))

    def add(self, a, b):
        return self.o.add(a, b)

    def add_plain(self, ct, vec):
        return self.o.add_pt(ct, self.o.encode(vec, ct.level, ct.scale))

    def rescale(self, ct):
        return self.o.rescale(ct)

    def level(self, ct):
        return ct.level


def _sum(be, terms):
    acc = None
    for t in terms:
        acc = t if acc is None else be.add(acc, t)
    return acc


# ---------------------------------------------------------------------------
# convolution (Section 4.1)
# ---------------------------------------------------------------------------

def _rotation_offsets(lam, need_b):
    """Block offsets r with, for each output block b, the input channel
    lam[b+r] it takes (indices mod the block count).  Every output block must
    see every channel present in the shard exactly once.  Phase 1 keeps the
    offsets that bring a new channel to every needed block at once (for
    consecutive d-fold copies these are 0, d, 2d, ...); phase 2 fills what is
    still missing block by block.  Smallest offset first in both phases."""
    nb = len(lam)
    chans = set(f for f in lam if f >= 0)
    covered = {b: set() for b in need_b}
    assign = {}
    for r in range(nb):
        fs = {b: lam[(b + r) % nb] for b in need_b}
        if all(f >= 0 and f not in covered[b] for b, f in fs.items()):
            assign[r] = fs
            for b, f in fs.items():
                covered[b].add(f)
    for r in range(nb):
        for b in need_b:
            f = lam[(b + r) % nb]
            if f >= 0 and f not in covered[b]:
                assign.setdefault(r, {})[b] = f
                covered[b].add(f)
    for b in need_b:
        if covered[b] != chans:
            raise ValueError("layout cannot be convolved")
    return [(r, assign[r]) for r in sorted(assign)]


def _tap_mask(lay, Ho, Wo, dk, dl):
    """Valid-output x valid-input mask of one block for the shift S_{dk,dl}."""
    mp = lay.mp
    i = np.arange(mp)[:, None]
    j = np.arange(mp)[None, :]
    m = (i < Ho) & (j < Wo) & (i + dk >= 0) & (i + dk < lay.H) & (j + dl >= 0) & (j + dl < lay.W)
    return m.astype(np.float64).reshape(-1)


def conv_plan(lay, w, pad):
    """Plan of a stride-1 convolution of an image-sharded input: the output
    layout and, per input shard u, the list of (rotation amount, {v: slot
    vector}) products.  Output shard v = sum over u and the list of
    pt * rot(ct_u, amount) (Section 4.1, single shard and image shards;
    duplicated / permuted inputs through the block map)."""
    out, plan = conv_plan_split(lay, w, pad)
    return out, [[(a, pts) for a, pts, _ in items] for items in plan]


def conv_plan_split(lay, w, pad):
    """conv_plan / conv_plan_channel with every amount split as
    (baby, giant): amount = baby + giant (mod N), baby the block offset r*B
    (0 for channel shards), giant the tap offset dk*mp + dl."""
    if lay.kind == "channel":
        out, plan = conv_plan_channel(lay, w, pad)
        return out, [[(a, pts, (0, a)) for a, pts in items] for items in plan]
    if lay.kind != "image":
        raise ValueError("image-shard layout expected")
    w = np.asarray(w, dtype=np.float64)
    Co, Ci, kh, kw = w.shape
    if Ci != lay.C:
        raise ValueError("channel mismatch")
    Ho, Wo = lay.H + 2 * pad - kh + 1, lay.W + 2 * pad - kw + 1
    if Ho < 1 or Wo < 1 or Ho > lay.mp or Wo > lay.mp:
        raise ValueError("bad convolution geometry")
    out = natural_layout(lay.N, Co, Ho, Wo, mp=lay.mp)
    if out.kind != "image":
        raise ValueError("output does not fit image shards")
    N, B, mp, nb = lay.N, lay.B, lay.mp, lay.nb
    need_b = [b for b in range(nb) if any(s[b] >= 0 for s in out.shards)]
    plan = []
    for u, lam in enumerate(lay.shards):
        items = []
        for r, fs in _rotation_offsets(lam, need_b):
            for kr in range(kh):
                for kc in range(kw):
                    dk, dl = kr - pad, kc - pad
                    mask = _tap_mask(lay, Ho, Wo, dk, dl)
                    if not mask.any():
                        continue
                    amount = (r * B + dk * mp + dl) % N
                    split = ((r * B) % N, (dk * mp + dl) % N)
                    pts = {}
                    for v, mu in enumerate(out.shards):
                        vec = BlockVec(N, B, mask)
                        for b, f in fs.items():
                            g = mu[b]
                            if g >= 0:
                                vec.set_block(b, w[g, f, kr, kc])
                        if vec.any():
                            pts[v] = vec
                    if pts:
                        items.append((amount, pts, split))
        plan.append(items)
    return out, plan


def conv_plan_channel(lay, w, pad):
    """Plan of a stride-1 convolution of a channel-sharded input (Section 4.1,
    "With Channel Shards"): shard (f, v) holds rows v*R .. v*R+R-1 of channel
    f (R = N/mp).  Every input shard is rotated cyclically by k*mp + l for each
    tap; output shard (g, v) takes, for each tap, the rows whose source row is
    in the same shard from rot([M^f]_v) (mask m) and the rows whose source row
    is in the neighbouring shard v + sign(k) from rot([M^f]_{v+sign k})
    (complementary mask); rows outside the channel read zero padding."""
    w = np.asarray(w, dtype=np.float64)
    Co, Ci, kh, kw = w.shape
    if Ci != lay.C:
        raise ValueError("channel mismatch")
    N, mp, H, W = lay.N, lay.mp, lay.H, lay.W
    R = N // mp
    spc = lay.B // N
    Ho, Wo = H + 2 * pad - kh + 1, W + 2 * pad - kw + 1
    if Ho < 1 or Wo < 1 or Ho > mp or Wo > mp:
        raise ValueError("bad convolution geometry")
    out = Layout(N, Co, Ho, Wo, mp, "channel", [(g, v) for g in range(Co) for v in range(spc)])
    out_index = {s: u for u, s in enumerate(out.shards)}
    il = np.arange(R)[:, None]
    jj = np.arange(mp)[None, :]
    plan = []
    for f, vin in lay.shards:
        items = []
        for kr in range(kh):
            for kc in range(kw):
                dk, dl = kr - pad, kc - pad
                amount = (dk * mp + dl) % N
                pts = {}
                # output shards that read this input shard for this tap: itself, and the shard
                # whose rows reach into this one (v = vin - sign(dk))
                cands = [vin] + ([vin - (1 if dk > 0 else -1)] if dk != 0 else [])
                for v in cands:
                    if v < 0 or v >= spc:
                        continue
                    gi = v * R + il                     # global output row
                    src = gi + dk                       # global source row
                    same = (il + dk >= 0) & (il + dk < R)
                    m = (gi < Ho) & (jj < Wo) & (src >= 0) & (src < H) & (jj + dl >= 0) & (jj + dl < W)
                    m = m & (same if v == vin else ~same)
                    if not m.any():
                        continue
                    mask = m.astype(np.float64).reshape(-1)
                    for g in range(Co):
                        wv = w[g, f, kr, kc]
                        if wv != 0.0:
                            pts[out_index[(g, v)]] = wv * mask
                if pts:
                    items.append((amount, pts))
        plan.append(items)
    return out, plan


def _accumulate_lazy(be, cts, nout, plan, pscale=None, rescale=True):
    """Lazy ModDown: every output shard v is
        (A0 + ModDown(E0), A1 + ModDown(E1)),
    E_p = sum over the nonzero rotations of pt * e_p (the key-switch product
    over Q and P, before ModDown), A0 = sum pt * sigma_g(c0) over those
    rotations plus pt * c0 over zero rotations, A1 = sum pt * c1 over zero
    rotations.  Same rotations and plaintexts as the per-rotation form; one
    ModDown per output shard instead of one per rotation.  Plaintexts are
    encoded at pscale (default q_level); rescale=False returns the sums."""
    o = be.o
    p = o.p
    lvl = cts[0].level
    if pscale is None:
        pscale = be.q(lvl)
    nq = lvl + 1
    qi, qpi = list(range(nq)), o.qp_index(lvl)
    nqp = len(qpi)
    E = [np.zeros((2, nqp, p.n), dtype=np.uint64) for _ in range(nout)]
    A = [np.zeros((2, nq, p.n), dtype=np.uint64) for _ in range(nout)]
    used = [False] * nout
    scale = None
    for u, items in enumerate(plan):
        if not items:
            continue
        ct = cts[u]
        ks = o.keyswitch_raw(ct, [a for a, _ in items])
        for e, (a, pts) in zip(ks, items):
            g = p.galois(a)
            for v, vec in pts.items():
                m = be.pt_coeffs(vec, pscale)
                ptq = o.limbs_of(m, lvl)
                used[v] = True
                scale = ct.scale * pscale
                if e is None:
                    for poly in range(2):
                        A[v][poly] = o.add_limbs(qi, A[v][poly], o.mul_limbs(qi, ptq, ct.data[poly]))
                else:
                    ptqp = o.limbs_qp(m, lvl)
                    for poly in range(2):
                        E[v][poly] = o.add_limbs(qpi, E[v][poly], o.mul_limbs(qpi, ptqp, e[poly]))
                    rc0 = o.automorph(qi, ct.data[0], g)
                    A[v][0] = o.add_limbs(qi, A[v][0], o.mul_limbs(qi, ptq, rc0))
    outs = []
    for v in range(nout):
        if not used[v]:
            raise ValueError("output shard without products")
        data = np.stack([o.add_limbs(qi, A[v][poly], o.moddown(lvl, E[v][poly])) for poly in range(2)])
        from .ckks import Ct
        ct = Ct(data, lvl, scale)
        outs.append(be.rescale(ct) if rescale else ct)
    return outs


def bsgs_split(steps, unit):
    """Baby / giant split of rotation amounts steps[t] = idx_t * unit: with
    G = ceil(sqrt(max idx + 1)), baby = (idx mod G) * unit and giant =
    (idx - idx mod G) * unit."""
    idx = [a // unit for a in steps]
    if any(i * unit != a for i, a in zip(idx, steps)):
        raise ValueError("amounts are not multiples of the unit")
    n = max(idx) + 1
    G = 1
    while G * G < n:
        G += 1
    return [((i % G) * unit, (i - i % G) * unit) for i in idx]


# masked sums of fewer rotations stay lazy in the baby-step / giant-step mode:
# below this size the ModUp/ModDown of the giant sums cost more than the key
# switches they save
BSGS_MIN_STEPS = 32


def _rot_masked_sums(be, ct, steps, masks, pscale, lazy=False, bsgs=False, unit=1):
    """Per output o: sum_t masks[o][t] * rot(ct, steps[t]) over the hoisted
    rotations of one ciphertext, not rescaled.  lazy (encrypted backend):
    the products are taken on the key-switch outputs over Q*P and each output
    takes one ModDown.  bsgs (encrypted backend): baby-step / giant-step over
    the split of bsgs_split(steps, unit), as in _conv_bsgs, when there are at
    least BSGS_MIN_STEPS amounts (lazy otherwise)."""
    if bsgs and len(steps) < BSGS_MIN_STEPS:
        bsgs, lazy = False, True
    if bsgs and isinstance(be, CkksBackend):
        split = bsgs_split(steps, unit)
        plan = [[(a, {o: m[t] for o, m in enumerate(masks)}, split[t]) for t, a in enumerate(steps)]]
        return _conv_bsgs(be, [ct], len(masks), plan, pscale=pscale, rescale=False)
    if lazy and isinstance(be, CkksBackend):
        plan = [[(a, {o: m[t] for o, m in enumerate(masks)}) for t, a in enumerate(steps)]]
        return _accumulate_lazy(be, [ct], len(masks), plan, pscale=pscale, rescale=False)
    rots = be.rotate_hoisted(ct, steps)
    return [_sum(be, [be.mul_plain(rots[t], m[t], pscale) for t in range(len(steps))]) for m in masks]


def _lazy_rotation_sum(be, terms):
    """sum of rot(ct, amount) over terms [(ct, amount)] of ciphertexts at one
    level and scale, with lazy ModDown: A + ModDown(E), E the sum of the
    key-switch products over Q and P, A the sum of sigma_g(c0) (and of the
    whole ciphertext for a rotation by zero)."""
    o = be.o
    p = o.p
    lvl = terms[0][0].level
    qi, qpi = list(range(lvl + 1)), o.qp_index(lvl)
    E = np.zeros((2, len(qpi), p.n), dtype=np.uint64)
    A = np.zeros((2, lvl + 1, p.n), dtype=np.uint64)
    for ct, a in terms:
        if ct.level != lvl or ct.scale != terms[0][0].scale:
            raise ValueError("rotation sum over different levels or scales")
        e = o.keyswitch_raw(ct, [a])[0]
        if e is None:
            for poly in range(2):
                A[poly] = o.add_limbs(qi, A[poly], ct.data[poly])
        else:
            for poly in range(2):
                E[poly] = o.add_limbs(qpi, E[poly], e[poly])
            A[0] = o.add_limbs(qi, A[0], o.automorph(qi, ct.data[0], p.galois(a)))
    from .ckks import Ct
    data = np.stack([o.add_limbs(qi, A[poly], o.moddown(lvl, E[poly])) for poly in range(2)])
    return Ct(data, lvl, terms[0][0].scale)


def _conv_bsgs(be, cts, nout, plan, pscale=None, rescale=True):
    """Baby-step / giant-step convolution with double hoisting.  Every amount
    is baby + giant (block offset + tap offset), and
        pt * rot_{b+g}(ct) = rot_g(roll(pt, g) * rot_b(ct)),
    so that, per giant g and output v,
        T_{g,v} = sum over inputs u and babies b of roll(pt, g) * rot_b(ct_u)
    is formed with lazy ModDown from the hoisted baby rotations of each input
    (one ModDown per (g, v)), and
        out_v = sum_g rot_g(T_{g,v})
    takes one key switch per (g, v) and one more lazy ModDown.  Rotations:
    (babies per input) + (giants x outputs) instead of one per amount."""
    if getattr(be, "basis", None) is not None:
        raise ValueError("basis-mask plaintexts are not taken by the baby-step/giant-step form")
    keys = sorted({(g, v) for items in plan for _, pts, (_, g) in items for v in pts})
    kidx = {k: i for i, k in enumerate(keys)}
    baby_plan = []
    for items in plan:
        byb = {}
        for _, pts, (b, g) in items:
            for v, vec in pts.items():
                byb.setdefault(b, {})[kidx[(g, v)]] = np.roll(vec, g)
        baby_plan.append(sorted(byb.items()))
    T = _accumulate_lazy(be, cts, len(keys), baby_plan, pscale=pscale, rescale=False)
    outs = []
    for v in range(nout):
        terms = [(T[kidx[(g, vv)]], g) for g, vv in keys if vv == v]
        if not terms:
            raise ValueError("output shard without products")
        o = _lazy_rotation_sum(be, terms)
        outs.append(be.rescale(o) if rescale else o)
    return outs


def conv2d(be, cts, lay, w, pad=1, stride=1, lazy=False, bsgs=False):
    """Homomorphic conv2d (cross-correlation, zero padding) of an image- or
    channel-sharded input; stride 2 is the stride-1 convolution followed by the
    downsampling step of the pooling (Section 4.1, strided convolution
    paragraph).  lazy=True accumulates the plaintext products before ModDown;
    bsgs=True evaluates the same sum by baby and giant steps (_conv_bsgs);
    both for the encrypted backend only (the slot simulator computes the same
    values either way), both with lazy downsampling for stride 2."""
    out_lay, split = conv_plan_split(lay, w, pad)
    plan = [[(a, pts) for a, pts, _ in items] for items in split]
    if bsgs and isinstance(be, CkksBackend):
        outs = _conv_bsgs(be, cts, len(out_lay.shards), split)
        if stride == 1:
            return outs, out_lay
        if stride != 2:
            raise ValueError("stride must be 1 or 2")
        return downsample_and_merge(be, outs, out_lay, select=True, bsgs=True)
    if lazy and isinstance(be, CkksBackend):
        outs = _accumulate_lazy(be, cts, len(out_lay.shards), plan)
        if stride == 1:
            return outs, out_lay
        if stride != 2:
            raise ValueError("stride must be 1 or 2")
        return downsample_and_merge(be, outs, out_lay, select=True, lazy=True)
    acc = [[] for _ in out_lay.shards]
    for u, items in enumerate(plan):
        if not items:
            continue
        lvl = be.level(cts[u])
        rots = be.rotate_hoisted(cts[u], [a for a, _ in items])
        for rot, (a, pts) in zip(rots, items):
            for v, vec in pts.items():
                acc[v].append(be.mul_plain(rot, vec, be.q(lvl)))
    outs = [be.rescale(_sum(be, terms)) for terms in acc]
    if stride == 1:
        return outs, out_lay
    if stride != 2:
        raise ValueError("stride must be 1 or 2")
    return downsample_and_merge(be, outs, out_lay, select=True)


# ---------------------------------------------------------------------------
# average pooling (Section 4.2)
# ---------------------------------------------------------------------------

def _hmask(lay, i, val):
    """rot_i of the mask that keeps column 2i of the even rows (valid blocks)."""
    blk = np.zeros((lay.mp, lay.mp))
    blk[0:lay.H:2, i] = val
    return _per_block(lay, blk)


def _vmask(lay, j, Wo):
    """rot_{3j mp/2} of the mask that keeps the left half of row 2j."""
    blk = np.zeros(lay.B)
    o = j * lay.mp // 2
    blk[o:o + Wo] = 1.0
    return _per_block(lay, blk.reshape(lay.mp, lay.mp))


def _fmask(lay, i, j, val):
    """Fused one-level mask: element (2j, 2i) of each block, after rot_i."""
    blk = np.zeros((lay.mp, lay.mp))
    blk[2 * j, i] = val
    return _per_block(lay, blk)


def _per_block(lay, blk, lam=None):
    """Repeat a block pattern over the blocks that hold a channel (any shard)."""
    v = np.zeros(lay.N)
    flat = blk.reshape(-1)
    valid = [any(s[b] >= 0 for s in lay.shards) for b in range(lay.nb)]
    for b in range(lay.nb):
        if valid[b]:
            v[b * lay.B:(b + 1) * lay.B] = flat
    return v


def downsample(be, cts, lay, select=False, fused=None, lazy=False, bsgs=False):
    """Per-shard downsample: (pool) 2x2 window sums, then horizontal and
    vertical reduction; (select) the reductions alone keep the top-left element
    of every 2x2 window (strided convolution).  Returns the shards with an
    (H/2 x W/2) channel packed at the start of every old block."""
    mp = lay.mp
    if select:
        Ho, Wo, val = (lay.H + 1) // 2, (lay.W + 1) // 2, 1.0
    else:
        if lay.H % 2 or lay.W % 2:
            raise ValueError("average pooling needs even H and W")
        Ho, Wo, val = lay.H // 2, lay.W // 2, 0.25
    outs = []
    for ct in cts:
        lvl = be.level(ct)
        if fused is None:
            use_fused = lvl < 2
        else:
            use_fused = fused
        if lvl < 1:
            raise ValueError("pooling needs a level")
        if not select:
            r = be.rotate_hoisted(ct, [1, mp, mp + 1])
            D = _sum(be, [ct] + r)
        else:
            D = ct
        hs = list(range(Wo))
        if use_fused:
            ps = be.q(lvl) / 4.0
            T = _rot_masked_sums(be, D, hs, [[_fmask(lay, i, j, val) for i in hs] for j in range(Ho)], ps, lazy,
                                 bsgs)
            moved = [T[0]] + [be.rotate(T[j], 3 * j * mp // 2) for j in range(1, Ho)]
            outs.append(be.rescale(_sum(be, moved)))
        else:
            M1 = be.rescale(_rot_masked_sums(be, D, hs, [[_hmask(lay, i, val) for i in hs]], be.q(lvl), lazy,
                                             bsgs)[0])
            lvl1 = be.level(M1)
            if lvl1 < 1:
                raise ValueError("separable pooling needs two levels")
            vs = [3 * j * mp // 2 for j in range(Ho)]
            outs.append(be.rescale(_rot_masked_sums(be, M1, vs, [[_vmask(lay, j, Wo) for j in range(Ho)]],
                                                    be.q(lvl1), lazy, bsgs, 3 * mp // 2)[0]))
    nl = Layout(lay.N, lay.C, Ho, Wo, mp // 2, "image",
                [[s[b // 4] if b % 4 == 0 else -1 for b in range(4 * lay.nb)] for s in lay.shards])
    return outs, nl


def consolidate(be, cts, lay):
    """Merge every four consecutive downsampled shards into one,
    S = S0 + S1>>q + S2>>2q + S3>>3q, q the post-pool block size: shard e of a
    group moves right by e (new) blocks.  Two shards give two summands and one
    shard none (Section 4.2, consolidation)."""
    t = len(cts)
    Bn = lay.B  # new (post-pool) block size; data sits at block 4b of each shard
    if t == 1:
        return cts, lay
    outs, maps = [], []
    for s0 in range(0, t, 4):
        g = min(4, t - s0)   # the last group may be short when t is not a multiple of 4
        terms = [cts[s0]] + [be.rotate(cts[s0 + e], -e * Bn) for e in range(1, g)]
        outs.append(_sum(be, terms))
        lam = [-1] * lay.nb
        for e in range(g):
            src = lay.shards[s0 + e]
            for b in range(lay.nb // 4):
                lam[4 * b + e] = src[4 * b]
        maps.append(lam)
    return outs, Layout(lay.N, lay.C, lay.H, lay.W, lay.mp, "image", maps)


def duplicate(be, ct, lay, d):
    """S' = S + S>>B' + ... (d summands, shifts by multiples of 4B'/d) for a
    single shard whose blocks 4b+e (e < 4/d) hold data (Section 4.2,
    duplication)."""
    Bn = lay.B
    step = 4 // d
    shifts = [-(c * step) * Bn for c in range(1, d)]
    rots = be.rotate_hoisted(ct, shifts)
    out = _sum(be, [ct] + rots)
    lam = list(lay.shards[0])
    for b in range(lay.nb // 4):
        for c in range(1, d):
            for e in range(step):
                lam[4 * b + c * step + e] = lam[4 * b + e]
    return out, Layout(lay.N, lay.C, lay.H, lay.W, lay.mp, "image", [lam])


def downsample_channel(be, cts, lay, select=False, fused=None, lazy=False, bsgs=False):
    """Channel shards are downsampled individually (Section 4.2, "With Channel
    Shards"): 2x2 sums stay inside a shard (R is even), column 2i of the even
    valid rows goes to column i, the left half of local row 2j to j*mp/2."""
    N, mp = lay.N, lay.mp
    R = N // mp
    if select:
        Wo, val = (lay.W + 1) // 2, 1.0
    else:
        if lay.H % 2 or lay.W % 2:
            raise ValueError("average pooling needs even H and W")
        Wo, val = lay.W // 2, 0.25
    outs = []
    for ct, (f, v) in zip(cts, lay.shards):
        lvl = be.level(ct)
        use_fused = (lvl < 2) if fused is None else fused
        if lvl < 1:
            raise ValueError("pooling needs a level")
        rows = [r for r in range(0, R, 2) if v * R + r < lay.H]   # even local rows of the channel
        js = [r // 2 for r in rows]
        if not js:
            # a shard below the channel's last row: its pooled content is zero
            z = be.rescale(be.mul_plain(ct, np.zeros(N), be.q(lvl) / 4.0 if use_fused else be.q(lvl)))
            if not use_fused:
                z = be.rescale(be.mul_plain(z, np.zeros(N), be.q(be.level(z))))
            outs.append(z)
            continue
        if not select:
            D = _sum(be, [ct] + be.rotate_hoisted(ct, [1, mp, mp + 1]))
        else:
            D = ct
        hs = list(range(Wo))

        def hmask(i):
            blk = np.zeros((R, mp))
            blk[rows, i] = val
            return blk.reshape(-1)

        def vmask(j):
            blk = np.zeros(N)
            blk[j * mp // 2: j * mp // 2 + Wo] = 1.0
            return blk

        def fmask(i, j):
            blk = np.zeros((R, mp))
            blk[2 * j, i] = val
            return blk.reshape(-1)

        if use_fused:
            ps = be.q(lvl) / 4.0
            T = _rot_masked_sums(be, D, hs, [[fmask(i, j) for i in hs] for j in js], ps, lazy, bsgs)
            moved = [T[0] if js[0] == 0 else be.rotate(T[0], 3 * js[0] * mp // 2)] + \
                    [be.rotate(T[t], 3 * j * mp // 2) for t, j in enumerate(js) if t > 0]
            outs.append(be.rescale(_sum(be, moved)))
        else:
            M1 = be.rescale(_rot_masked_sums(be, D, hs, [[hmask(i) for i in hs]], be.q(lvl), lazy, bsgs)[0])
            lvl1 = be.level(M1)
            if lvl1 < 1:
                raise ValueError("separable pooling needs two levels")
            vs = [3 * j * mp // 2 for j in js]
            outs.append(be.rescale(_rot_masked_sums(be, M1, vs, [[vmask(j) for j in js]], be.q(lvl1), lazy, bsgs,
                                                    3 * mp // 2)[0]))
    return outs


def merge_channel(be, outs, lay, H2, W2):
    """Consolidate every four consecutive downsampled channel shards (shifts by
    multiples of N/4); the result is channel-sharded again when a pooled
    channel still exceeds N slots, image-sharded otherwise.  One channel in two
    shards is duplicated by two.  No permutation arises."""
    N, mp = lay.N, lay.mp
    q = N // 4
    t = len(outs)
    res, groups = [], []
    for s0 in range(0, t, 4):
        g = min(4, t - s0)
        terms = [outs[s0]] + [be.rotate(outs[s0 + e], -e * q) for e in range(1, g)]
        res.append(_sum(be, terms))
        groups.append(lay.shards[s0:s0 + g])
    mp2 = mp // 2
    B2 = mp2 * mp2
    if B2 > N:
        shards = [(grp[0][0], grp[0][1] // 4) for grp in groups]
        return res, Layout(N, lay.C, H2, W2, mp2, "channel", shards)
    nb = N // B2                       # pooled channels per ciphertext
    per_ch = B2 // q                   # quarters per pooled channel
    maps = []
    for grp in groups:
        lam = [-1] * nb
        for e, (f, part) in enumerate(grp):
            lam[e // per_ch] = f
        maps.append(lam)
    out = Layout(N, lay.C, H2, W2, mp2, "image", maps)
    if t == 2:   # one channel in two shards: duplicate x2
        res = [_sum(be, [res[0], be.rotate(res[0], -N // 2)])]
        out = Layout(N, lay.C, H2, W2, mp2, "image", [[maps[0][0]] * nb])
    return res, out


def downsample_and_merge(be, cts, lay, select=False, fused=None, lazy=False, bsgs=False):
    """Downsample every shard, then consolidate and duplicate (Section 4.2);
    lazy: the masked rotation sums of the downsampling take one ModDown each;
    bsgs: they are evaluated by baby and giant steps."""
    if lay.kind == "channel":
        outs = downsample_channel(be, cts, lay, select=select, fused=fused, lazy=lazy, bsgs=bsgs)
        if select:
            H2, W2 = (lay.H + 1) // 2, (lay.W + 1) // 2
        else:
            H2, W2 = lay.H // 2, lay.W // 2
        return merge_channel(be, outs, lay, H2, W2)
    outs, nl = downsample(be, cts, lay, select=select, fused=fused, lazy=lazy, bsgs=bsgs)
    t = len(outs)
    if t == 1:
        o, l2 = duplicate(be, outs[0], nl, 4)
        return [o], l2
    outs, nl = consolidate(be, outs, nl)
    if t == 2:
        o, l2 = duplicate(be, outs[0], nl, 2)
        return [o], l2
    return outs, nl


def avgpool2x2(be, cts, lay, fused=None, lazy=False, bsgs=False):
    """2x2 average pooling: downsample, consolidate, duplicate (Section 4.2),
    for image shards and channel shards; lazy / bsgs as in downsample_and_merge."""
    return downsample_and_merge(be, cts, lay, select=False, fused=fused, lazy=lazy, bsgs=bsgs)


# ---------------------------------------------------------------------------
# linear and pool-linear layers (Section 4.3, "Linear")
# ---------------------------------------------------------------------------

def linear_vectors(lay, W, pool=False):
    """Per output o and shard u: the slot vector that multiplies shard u for
    output o (None where it is zero).  Linear: W is [O][C*H*W] over the input
    in [C][H][W] order; pool-linear: W is [O][C] and every valid position of
    channel f carries W[o][f] / (H*W) (the global average pool folded into the
    weights).  A channel held in several blocks (duplicated copies) is read
    from its first block in shard-then-block order only."""
    W = np.asarray(W, dtype=np.float64)
    O = W.shape[0]
    C, H, Wd, N, mp = lay.C, lay.H, lay.W, lay.N, lay.mp
    if pool:
        if W.shape[1] != C:
            raise ValueError("pool-linear weights must be [O][C]")
        Wf = np.repeat(W / float(H * Wd), H * Wd, axis=1).reshape(O, C, H, Wd)
    else:
        if W.shape[1] != C * H * Wd:
            raise ValueError("linear weights must be [O][C*H*W]")
        Wf = W.reshape(O, C, H, Wd)
    vecs = [[None] * len(lay.shards) for _ in range(O)]
    if lay.kind == "channel":
        R = N // mp
        for u, (f, part) in enumerate(lay.shards):
            rows = [r for r in range(R) if part * R + r < H]
            if not rows:
                continue
            for o in range(O):
                v = np.zeros(N)
                for r in rows:
                    v[r * mp: r * mp + Wd] = Wf[o, f, part * R + r]
                vecs[o][u] = v
        return vecs
    seen = set()
    place = []
    for u, lam in enumerate(lay.shards):
        for b, f in enumerate(lam):
            if f >= 0 and f not in seen:
                seen.add(f)
                place.append((u, b, f))
    if len(seen) != C:
        raise ValueError("channel missing from the layout")
    for o in range(O):
        for u, b, f in place:
            if vecs[o][u] is None:
                vecs[o][u] = np.zeros(N)
            blk = np.zeros((mp, mp))
            blk[:H, :Wd] = Wf[o, f]
            vecs[o][u][b * lay.B:(b + 1) * lay.B] = blk.reshape(-1)
    return vecs


def linear(be, cts, lay, W, pool=False):
    """Each output o: the products of the shards with its weight vectors are
    summed and rescaled, then summed over all slots by rotate-and-add with
    rotations N/2, N/4, ..., 1 (every slot then holds the dot product), and
    masked onto slot o; the masked outputs are summed into one ciphertext and
    rescaled.  Two levels; output o sits in slot o."""
    vecs = linear_vectors(lay, W, pool)
    N = lay.N
    outs = []
    for o, per_shard in enumerate(vecs):
        prods = [be.mul_plain(cts[u], v, be.q(be.level(cts[u]))) for u, v in enumerate(per_shard) if v is not None]
        acc = be.rescale(_sum(be, prods))
        k = N // 2
        while k >= 1:
            acc = be.add(acc, be.rotate(acc, k))
            k //= 2
        e = np.zeros(N)
        e[o] = 1.0
        outs.append(be.mul_plain(acc, e, be.q(be.level(acc))))
    return be.rescale(_sum(be, outs))


def ref_linear(x, W, pool=False):
    """FP64 reference: W @ x.flatten(), or W @ mean over H, W (pool-linear)."""
    x = np.asarray(x, dtype=np.float64)
    if pool:
        return np.asarray(W, dtype=np.float64) @ x.mean(axis=(1, 2))
    return np.asarray(W, dtype=np.float64) @ x.reshape(-1)


# ---------------------------------------------------------------------------
# polynomial activations in the Chebyshev basis (Section 4.3, GELU)
# ---------------------------------------------------------------------------

def cheb_divide(c, g):
    """p = q * T_g + r for p = sum_j c[j] T_j with g <= deg p < 2g, from
    T_j = 2 T_g T_{j-g} - T_{2g-j} (j > g): q[0] = c[g], q[j-g] = 2 c[j] and
    r[2g-j] -= c[j] for j > g; r starts as c[0..g-1].  Plain loops in
    ascending j, so that any implementation doing the same IEEE operations
    gets the same doubles."""
    d = len(c) - 1
    q = [0.0] * (d - g + 1)
    r = [float(x) for x in c[:g]]
    q[0] = float(c[g])
    for j in range(g + 1, d + 1):
        q[j - g] = 2.0 * float(c[j])
        r[2 * g - j] = r[2 * g - j] - float(c[j])
    return q, r


def cheb_baby_size(d):
    """Baby-step size m: the smallest power of two with m * m >= d + 1."""
    m = 1
    while m * m < d + 1:
        m *= 2
    return m


class ChebEval:
    """Evaluation of p(y) = sum_k c_k T_k(y), y = (2x - (a + b)) / (b - a),
    on an encrypted x (oracle ciphertexts).

    Map: on [a, b] = [-1, 1], y = x and no level is spent (an affine map in
    front of the activation folds into the preceding convolution's weights and
    bias, as batch normalization does, Sec. 4.3); otherwise y = alpha x + beta
    costs one constant product.

    Scales: every ciphertext at level l carries the nominal scale S[l], with
    S[l0] the input's scale and S[l-1] = S[l]^2 / q_l, so that the product
    of two level-l ciphertexts, rescaled, has exactly scale S[l-1].  A
    constant multiplies a level-l' operand (l' = l, or a ciphertext dropped
    to l) at S[l-1] q_l / (the operand's scale), which brings it to S[l-1]
    after the rescale; level adjustments drop limbs, then multiply by 1 in
    the same way.  Results are given the nominal scale of their level.

    Basis: T_1 = y, T_{2k} = 2 T_k^2 - 1, T_{2k+1} = 2 T_{k+1} T_k - T_1
    for k < m (m = cheb_baby_size(deg)), and the giant powers T_{2m},
    T_{4m}, ... by doubling (the recurrences of the Chebyshev polynomials in
    the Appendix, Polynomial Approximation).  A polynomial of degree < m is
    c_0 plus the sum of the constant products c_j T_j, each T_j dropped to one
    common level and the sum rescaled once; a larger one is split by
    cheb_divide at the largest giant power g <= deg and evaluated as
    q(y) T_g + r(y)."""

    def __init__(self, be, x, a, b):
        self.be, self.o = be, be.o
        self.S = {x.level: x.scale}
        l = x.level
        while l > 0:
            self.S[l - 1] = (self.S[l] * self.S[l]) / self.o.p.q[l]
            l -= 1
        self.a, self.b = float(a), float(b)
        self.x = x
        self._adj = {}

    def _const_mul_raw(self, ct, value):
        """ct (level l) * value at S[l-1] q_l / ct.scale, not rescaled; nominal
        scale S[l-1] q_l."""
        l = ct.level
        pscale = self.S[l - 1] * float(self.o.p.q[l]) / ct.scale
        r = self.o.mul_const(ct, value, pscale)
        return type(r)(r.data, r.level, self.S[l - 1] * float(self.o.p.q[l]))

    def _const_mul(self, ct, value):
        """ct (level l) * value -> level l-1, scale S[l-1]."""
        l = ct.level
        r = self.o.rescale(self._const_mul_raw(ct, value))
        return type(r)(r.data, r.level, self.S[l - 1])

    def adjust(self, ct, level):
        """ct brought down to `level` (a cached result per ciphertext and level)."""
        if ct.level == level:
            return ct
        if ct.level < level:
            raise ValueError("cannot raise a level")
        key = (id(ct), level)
        if key not in self._adj:
            self._adj[key] = (ct, self._const_mul(self.o.drop_to(ct, level + 1), 1.0))
        return self._adj[key][1]

    def mul(self, u, v):
        l = min(u.level, v.level)
        u, v = self.adjust(u, l), self.adjust(v, l)
        r = self.o.rescale(self.o.mul_ct(u, v))
        assert r.scale == self.S[l - 1]
        return r

    def add(self, u, v):
        l = min(u.level, v.level)
        return self.o.add(self.adjust(u, l), self.adjust(v, l))

    def affine(self):
        """y = alpha x + beta, alpha = 2 / (b - a), beta = -(a + b) / (b - a);
        y = x on [-1, 1]."""
        if self.a == -1.0 and self.b == 1.0:
            return self.x
        alpha = 2.0 / (self.b - self.a)
        beta = -(self.a + self.b) / (self.b - self.a)
        y = self._const_mul(self.x, alpha)
        return self.o.add_const(y, beta)

    def basis(self, y, m, d):
        T = {1: y}
        for k in range(2, min(m, d + 1)):
            if k % 2 == 0:
                p = self.mul(T[k // 2], T[k // 2])
                T[k] = self.o.add_const(self.o.add(p, p), -1.0)
            else:
                h = k // 2
                p = self.mul(T[h + 1], T[h])
                T[k] = self.o.sub(self.o.add(p, p), self.adjust(T[1], p.level))
        g = m
        while g <= d:
            h = g // 2
            p = self.mul(T[h], T[h])
            T[g] = self.o.add_const(self.o.add(p, p), -1.0)
            g *= 2
        return T

    def lin(self, c, T):
        """c[0] + sum_j c[j] T_j (j >= 1, c[j] != 0): every T_j dropped to the
        level above the lowest one's, multiplied by c[j], summed, rescaled
        once; a plain float when no c[j], j >= 1, is nonzero."""
        js = [j for j in range(1, len(c)) if c[j] != 0.0]
        if not js:
            return float(c[0])
        top = min(T[j].level for j in js) - 1
        if top < 0:
            raise ValueError("out of levels")
        acc = None
        for j in js:
            t = self._const_mul_raw(self.o.drop_to(T[j], top + 1), c[j])
            acc = t if acc is None else self.o.add(acc, t)
        r = self.o.rescale(acc)
        r = type(r)(r.data, r.level, self.S[top])
        return self.o.add_const(r, c[0]) if c[0] != 0.0 else r

    def _sum(self, u, v):
        """u + v where either may be a plain float."""
        if isinstance(u, float) and isinstance(v, float):
            return u + v
        if isinstance(u, float):
            u, v = v, u
        if isinstance(v, float):
            return self.o.add_const(u, v) if v != 0.0 else u
        return self.add(u, v)

    def ev(self, c, T, m):
        d = len(c) - 1
        if d < m:
            return self.lin(c, T)
        g = m
        while 2 * g <= d:
            g *= 2
        q, r = cheb_divide(c, g)
        Q = self.ev(q, T, m)
        if isinstance(Q, float):
            P = self._const_mul(T[g], Q) if Q != 0.0 else 0.0
        else:
            P = self.mul(Q, T[g])
        R = self.ev(r, T, m)
        return self._sum(P, R)

    def run(self, coeffs):
        c = [float(v) for v in coeffs]
        d = len(c) - 1
        if d < 1:
            raise ValueError("degree must be at least 1")
        m = cheb_baby_size(d)
        y = self.affine()
        T = self.basis(y, m, d)
        r = self.ev(c, T, m)
        if isinstance(r, float):
            raise ValueError("constant polynomial")
        return r


def cheb_eval(be, ct, coeffs, a, b):
    """Encrypted p(x) = sum_k coeffs[k] T_k((2x - a - b)/(b - a)) (ChebEval)."""
    return ChebEval(be, ct, a, b).run(coeffs)


def ref_cheb(x, coeffs, a, b):
    """FP64 reference of the same polynomial."""
    y = (2.0 * np.asarray(x, dtype=np.float64) - (a + b)) / (b - a)
    return np.polynomial.chebyshev.chebval(y, np.asarray(coeffs, dtype=np.float64))


# ---------------------------------------------------------------------------
# bias, batch-norm folding and the basic block (Section 4.3)
# ---------------------------------------------------------------------------

def add_bias(be, cts, lay, bias):
    """Per-channel bias: the plaintext of an image whose channel f is bias[f]
    on every valid pixel (packed like the input), added to every shard."""
    bias = np.asarray(bias, dtype=np.float64)
    x = np.broadcast_to(bias[:, None, None], (lay.C, lay.H, lay.W))
    return [be.add_plain(ct, v) for ct, v in zip(cts, pack(x, lay))]


def fold_bn(w, gamma, shift, div=1.0):
    """Inference batch norm y = gamma * conv(x, w) + shift folded into the
    convolution (Section 4.3, Batch Normalization), and the result divided by
    div (the map of [-div, div] onto [-1, 1] in front of the activation):
    weights w[o] * (gamma[o] / div), bias shift[o] / div."""
    w = np.asarray(w, dtype=np.float64)
    s = np.asarray(gamma, dtype=np.float64) / float(div)
    return w * s[:, None, None, None], np.asarray(shift, dtype=np.float64) / float(div)


def basic_block(be, cts, lay, w1, bn1, w2, bn2, bound, coeffs, lazy=False, bsgs=False):
    """conv(w1) with batch norm bn1 = (gamma, shift) folded and divided by the
    activation bound -> GELU as the Chebyshev series coeffs on [-1, 1] (the
    expansion of GELU(bound * y)) -> conv(w2) with bn2 folded -> 2x2 average
    pooling; same padding (k // 2), stride 1.  bn2 may be None (no bias)."""
    k = np.asarray(w1).shape[2]
    w1f, b1f = fold_bn(w1, bn1[0], bn1[1], bound)
    cts, lay = conv2d(be, cts, lay, w1f, pad=k // 2, stride=1, lazy=lazy, bsgs=bsgs)
    cts = add_bias(be, cts, lay, b1f)
    cts = [ChebEval(be, ct, -1.0, 1.0).run(coeffs) for ct in cts]
    k2 = np.asarray(w2).shape[2]
    if bn2 is None:
        w2f = np.asarray(w2, dtype=np.float64)
    else:
        w2f, b2f = fold_bn(w2, bn2[0], bn2[1], 1.0)
    cts, lay = conv2d(be, cts, lay, w2f, pad=k2 // 2, stride=1, lazy=lazy, bsgs=bsgs)
    if bn2 is not None:
        cts = add_bias(be, cts, lay, b2f)
    return avgpool2x2(be, cts, lay, lazy=lazy, bsgs=bsgs)


def ref_basic_block(x, w1, bn1, w2, bn2, bound, coeffs):
    """FP64 reference of basic_block (the activation as the same polynomial)."""
    k, k2 = np.asarray(w1).shape[2], np.asarray(w2).shape[2]
    u = ref_conv2d(x, w1, pad=k // 2) * np.asarray(bn1[0])[:, None, None] + np.asarray(bn1[1])[:, None, None]
    a = ref_cheb(u / bound, coeffs, -1.0, 1.0)
    v = ref_conv2d(a, w2, pad=k2 // 2)
    if bn2 is not None:
        v = v * np.asarray(bn2[0])[:, None, None] + np.asarray(bn2[1])[:, None, None]
    return ref_avgpool2x2(v)


# ---------------------------------------------------------------------------
# FP64 references (PyTorch semantics)
# ---------------------------------------------------------------------------

def ref_conv2d(x, w, pad=1, stride=1):
    """Direct FP64 cross-correlation with zero padding (the paper's Eq. (1))."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    C, H, W = x.shape
    Co, Ci, kh, kw = w.shape
    xp = np.zeros((C, H + 2 * pad, W + 2 * pad))
    xp[:, pad:pad + H, pad:pad + W] = x
    Ho, Wo = H + 2 * pad - kh + 1, W + 2 * pad - kw + 1
    out = np.zeros((Co, Ho, Wo))
    for a in range(kh):
        for b in range(kw):
            out += np.einsum("gf,fij->gij", w[:, :, a, b], xp[:, a:a + Ho, b:b + Wo])
    return out[:, ::stride, ::stride]


def ref_avgpool2x2(x):
    C, H, W = x.shape
    return x[:, : H // 2 * 2, : W // 2 * 2].reshape(C, H // 2, 2, W // 2, 2).mean(axis=(2, 4))
