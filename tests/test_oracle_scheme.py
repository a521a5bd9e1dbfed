"""Pins of the oracle's RNS-CKKS scheme steps (CPU only).

* ModUp (fast base conversion) vs big-integer CRT: every output residue is
  (X + u*D) mod t for one u in [0, alpha), X the digit's CRT value;
* ModDown vs big integers: output = floor(X / P) - u for one u in [0, k);
* rescale vs big integers: output = (X - [X]_{q_l}) / q_l exactly, with the
  centered residue;
* encryption/decryption within the fresh-noise bound;
* rotation commutes with decryption as np.roll; rotation by 0 is the identity;
  rotations compose; hoisted and one-at-a-time rotations agree bit for bit;
* plaintext product + rescale decrypts to the slot-wise product.
"""
import numpy as np
import pytest

from oracle import ckks


def crt(res, mods):
    Q = 1
    for q in mods:
        Q *= q
    x = 0
    for r, q in zip(res, mods):
        Qi = Q // q
        x += int(r) * Qi * pow(Qi % q, -1, q)
    return x % Q, Q


@pytest.fixture(scope="module")
def small():
    p = ckks.Params(5, [50, 40, 40, 40, 40], [55, 55], 2)   # alpha = 3: digits {0,1,2}, {3,4}
    return p, ckks.Oracle(p, 77)


def test_modup_bigint(small):
    p, o = small
    rng = np.random.default_rng(0)
    level = 4
    x = np.stack([rng.integers(0, q, p.n, dtype=np.uint64) for q in p.q[: level + 1]])
    nqp = level + 1 + p.k
    mods = p.q[: level + 1] + p.p
    for j in range((level + p.alpha) // p.alpha):
        out = np.zeros((nqp, p.n), dtype=np.uint64)
        ckks.lib().orc_modup(p.cref, level, j, ckks.ptr(x), ckks.ptr(out))
        digit = list(range(j * p.alpha, min((j + 1) * p.alpha, level + 1)))
        dm = [p.q[i] for i in digit]
        for c in range(p.n):
            X, D = crt([x[i, c] for i in digit], dm)
            us = set()
            for o_, t in enumerate(mods):
                if o_ in digit:
                    assert out[o_, c] == x[o_, c]
                    continue
                cand = [u for u in range(len(digit)) if (X + u * D) % t == int(out[o_, c])]
                assert cand, (j, c, o_)
                us.add(cand[0])
            assert len(us) <= 1   # one lift u for the whole coefficient


def test_moddown_bigint(small):
    p, o = small
    rng = np.random.default_rng(1)
    level = 3
    mods = p.q[: level + 1] + p.p
    x = np.stack([rng.integers(0, q, p.n, dtype=np.uint64) for q in mods])
    out = np.zeros((level + 1, p.n), dtype=np.uint64)
    ckks.lib().orc_moddown(p.cref, level, ckks.ptr(x), ckks.ptr(out))
    P = 1
    for t in p.p:
        P *= t
    for c in range(p.n):
        X, _ = crt([x[i, c] for i in range(len(mods))], mods)
        base = X // P
        cand = [u for u in range(p.k) if all((base - u) % p.q[i] == int(out[i, c]) for i in range(level + 1))]
        assert cand, c


def test_moddown_absorbs_multiples_of_P(med):
    """ModDown(e + P a) = ModDown(e) + a exactly, for any e over Q_l and P and
    any a over Q_l (P a is zero on the special primes, so the conversion of
    the P part is unchanged, and the division by P returns a): the identity
    that lets a hoisted rotation add P * sigma_g(c0) to its key-switch product
    instead of adding sigma_g(c0) after the ModDown."""
    p, o = med
    rng = np.random.default_rng(11)
    for level in (0, 2, 5):
        mods = p.q[: level + 1] + p.p
        e = np.stack([rng.integers(0, q, p.n, dtype=np.uint64) for q in mods])
        a = np.stack([rng.integers(0, q, p.n, dtype=np.uint64) for q in p.q[: level + 1]])
        P = 1
        for t in p.p:
            P *= t
        ePa = e.copy()
        for i, q in enumerate(p.q[: level + 1]):
            ePa[i] = np.array([(int(x) + int(y) * (P % q)) % q for x, y in zip(e[i], a[i])], dtype=np.uint64)
        lhs = o.moddown(level, ePa)
        base = o.moddown(level, e)
        rhs = np.stack([np.array([(int(x) + int(y)) % q for x, y in zip(base[i], a[i])], dtype=np.uint64)
                        for i, q in enumerate(p.q[: level + 1])])
        assert (lhs == rhs).all(), level


def test_rescale_bigint(small):
    p, o = small
    rng = np.random.default_rng(2)
    level = 4
    ct = np.stack([np.stack([rng.integers(0, q, p.n, dtype=np.uint64) for q in p.q[: level + 1]])
                   for _ in range(2)])
    out = np.zeros((2, level, p.n), dtype=np.uint64)
    ckks.lib().orc_rescale(p.cref, level, ckks.ptr(ct), ckks.ptr(out))
    ql = p.q[level]
    for poly in range(2):
        for c in range(p.n):
            X, _ = crt([ct[poly, i, c] for i in range(level + 1)], p.q[: level + 1])
            r = X % ql
            if r > (ql - 1) // 2:
                r -= ql
            y = (X - r) // ql
            assert (X - r) % ql == 0
            for i in range(level):
                assert int(out[poly, i, c]) == y % p.q[i]


@pytest.fixture(scope="module")
def med():
    p = ckks.Params(10, [60, 40, 40, 40, 40, 40], [60, 60], 3)
    return p, ckks.Oracle(p, 123)


def test_encrypt_decrypt(med):
    p, o = med
    z = np.random.default_rng(4).uniform(-1, 1, p.N)
    for level in (0, 2, 5):
        ct = o.encrypt(o.encode(z, level, 2.0 ** 40), seed=9, index=level)
        assert ct.data.shape == (2, level + 1, p.n)
        assert np.abs(o.decrypt(ct) - z).max() < 1e-7


def test_encrypt_is_deterministic_and_drops_limbs(med):
    p, o = med
    z = np.random.default_rng(5).uniform(-1, 1, p.N)
    pt5 = o.encode(z, 5, 2.0 ** 40)
    a = o.encrypt(pt5, seed=3, index=1)
    b = o.encrypt(pt5, seed=3, index=1)
    assert (a.data == b.data).all()
    c = o.encrypt(o.encode(z, 2, 2.0 ** 40), seed=3, index=1)
    assert (c.data == a.data[:, :3]).all()
    d = o.encrypt(pt5, seed=3, index=2)
    assert not (d.data == a.data).all()


def test_rotation_invariants(med):
    p, o = med
    z = np.random.default_rng(6).uniform(-1, 1, p.N)
    ct = o.encrypt(o.encode(z, 4, 2.0 ** 40), seed=1)
    steps = [1, 2, 5, p.N - 1, -3, 64, 0]
    rots = o.rotate_hoisted(ct, steps)
    for r, rc in zip(steps, rots):
        assert np.abs(o.decrypt(rc) - np.roll(z, -r)).max() < 1e-6
    assert (rots[-1].data == ct.data).all()
    # one at a time == hoisted, bit for bit (ModUp precedes the automorphism)
    for r, rc in zip(steps[:3], rots[:3]):
        assert (o.rotate(ct, r).data == rc.data).all()
    # composition
    r2 = o.rotate(o.rotate(ct, 3), 5)
    assert np.abs(o.decrypt(r2) - np.roll(z, -8)).max() < 1e-6
    # lower levels (partial last digit, single digit)
    for level in (0, 1, 3):
        c2 = o.drop_to(ct, level)
        assert np.abs(o.decrypt(o.rotate(c2, 7)) - np.roll(z, -7)).max() < 1e-6


def test_mul_pt_rescale_add(med):
    p, o = med
    rng = np.random.default_rng(7)
    z, w = rng.uniform(-1, 1, p.N), rng.uniform(-1, 1, p.N)
    lvl = 5
    ct = o.encrypt(o.encode(z, lvl, 2.0 ** 40), seed=2)
    pt = o.encode(w, lvl, float(p.q[lvl]))
    prod = o.rescale(o.mul_pt(ct, pt))
    assert prod.level == lvl - 1 and prod.scale == 2.0 ** 40
    assert np.abs(o.decrypt(prod) - z * w).max() < 1e-6
    s = o.add(prod, prod)
    assert np.abs(o.decrypt(s) - 2 * z * w).max() < 1e-6
    with pytest.raises(ValueError):
        o.add(prod, ct)


def negacyclic(a, b, q):
    """Schoolbook product in Z_q[x]/(x^n + 1) with Python integers."""
    n = len(a)
    out = [0] * n
    for i in range(n):
        ai = int(a[i])
        if ai == 0:
            continue
        for j in range(n):
            k = i + j
            if k < n:
                out[k] += ai * int(b[j])
            else:
                out[k - n] -= ai * int(b[j])
    return [v % q for v in out]


def test_keyswitch_raw_pins(small):
    """The key-switch product before ModDown (lazy ModDown's building block):
    (1) it is sum_j sigma_g(ModUp_j(c1)) * swk_{g,j} over Q_l and P, recomputed
    with the schoolbook negacyclic product and Python integers; (2) ModDown of
    it plus sigma_g(c0) is the rotation itself, bit for bit, at full and
    partial-digit levels."""
    p, o = small
    rng = np.random.default_rng(11)
    z = rng.uniform(-1, 1, p.N)
    for level in (4, 2):
        ct = o.encrypt(o.encode(z, level, 2.0 ** 30), seed=5, index=level)
        steps = [1, 3, -2]
        raw = o.keyswitch_raw(ct, steps)
        rots = o.rotate_hoisted(ct, steps)
        qp = o.qp_index(level)
        nqp = len(qp)
        beta = (level + p.alpha) // p.alpha
        D = []
        for j in range(beta):
            out = np.zeros((nqp, p.n), dtype=np.uint64)
            ckks.lib().orc_modup(p.cref, level, j, ckks.ptr(np.ascontiguousarray(ct.data[1])), ckks.ptr(out))
            D.append(out)
        for s, e, rc in zip(steps, raw, rots):
            g = p.galois(s)
            kc = o.swk(g)[0]                     # coefficient form [dnum][2][L+1+k][n]
            for o_, pi in enumerate(qp):
                q = p.mod[pi]
                acc0, acc1 = [0] * p.n, [0] * p.n
                for j in range(beta):
                    d = o.automorph([pi], D[j][o_:o_ + 1], g)[0]
                    acc0 = [(x + y) % q for x, y in zip(acc0, negacyclic(d, kc[j][0][pi], q))]
                    acc1 = [(x + y) % q for x, y in zip(acc1, negacyclic(d, kc[j][1][pi], q))]
                assert [int(v) for v in e[0][o_]] == acc0, (level, s, pi)
                assert [int(v) for v in e[1][o_]] == acc1, (level, s, pi)
            qi = list(range(level + 1))
            c0g = o.automorph(qi, ct.data[0], g)
            f0 = o.add_limbs(qi, c0g, o.moddown(level, e[0]))
            f1 = o.moddown(level, e[1])
            assert (f0 == rc.data[0]).all() and (f1 == rc.data[1]).all(), (level, s)


def test_keygen_limb_subset(med):
    """Keys generated on a subset of the primes (for low-level tests of large
    parameter sets) equal the full keys on those limbs, and rotations with
    them equal rotations with the full keys bit for bit."""
    p, o = med
    g = p.galois(3)
    full = o.swk(g)[0]
    pidx = o.qp_index(2)
    sub = o.swk_limbs_coeff(g, pidx)
    assert (sub[:, :, pidx, :] == full[:, :, pidx, :]).all()
    others = [i for i in range(p.L + 1 + p.k) if i not in pidx]
    assert not sub[:, :, others, :].any()
    o2 = ckks.Oracle(p, o.seed, key_level=2)
    z = np.random.default_rng(8).uniform(-1, 1, p.N)
    ct = o.encrypt(o.encode(z, 2, 2.0 ** 40), seed=6)
    for a, b in zip(o.rotate_hoisted(ct, [3, 1]), o2.rotate_hoisted(ct, [3, 1])):
        assert (a.data == b.data).all()
    with pytest.raises(ValueError):
        o2.rotate(o.encrypt(o.encode(z, 3, 2.0 ** 40), seed=6), 3)
