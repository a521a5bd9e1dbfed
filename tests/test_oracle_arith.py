"""Pins of the oracle's integer layer against closed forms, brute force and
published test vectors (CPU only).

* modular product / power / inverse vs Python big integers;
* primality vs trial division and known pseudoprimes;
* the prime chain (first prime 2^b - j*2n + 1, skipping taken ones) vs an
  independent Python search;
* the negacyclic NTT vs direct evaluation at psi^(2k+1) and the polynomial
  product vs the schoolbook negacyclic product;
* ChaCha20 vs RFC 8439 test vectors; samplers' word-to-coefficient mapping and
  their distributions.
"""
import ctypes
import math
import os

import numpy as np
import pytest

from oracle import ckks

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def py_is_prime(m):
    if m < 2:
        return False
    if m < 1 << 20:
        return all(m % d for d in range(2, int(math.isqrt(m)) + 1))
    # an independent Miller-Rabin with Python integers and different bases
    d, s = m - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 325, 9375, 28178, 450775, 9780504, 1795265022):
        a %= m
        if a == 0:
            continue
        x = pow(a, d, m)
        if x in (1, m - 1):
            continue
        for _ in range(s - 1):
            x = x * x % m
            if x == m - 1:
                break
        else:
            return False
    return True


def test_mulmod_powmod_invmod():
    L = ckks.lib()
    rng = np.random.default_rng(1)
    for bits in (20, 40, 50, 60, 61):
        q = int(L.orc_find_prime(bits, 1024, None, 0))
        for _ in range(200):
            a, b = int(rng.integers(0, q)), int(rng.integers(0, q))
            assert L.orc_mulmod(a, b, q) == a * b % q
            e = int(rng.integers(0, 1 << 62))
            assert L.orc_powmod(a, e, q) == pow(a, e, q)
            if a:
                assert L.orc_invmod(a, q) * a % q == 1


def test_is_prime():
    L = ckks.lib()
    for m in range(0, 3000):
        assert bool(L.orc_is_prime(m)) == py_is_prime(m), m
    # Carmichael numbers and strong pseudoprimes to small base sets
    for m in (561, 1105, 41041, 825265, 3215031751, 2152302898747, 3474749660383, 341550071728321,
              3825123056546413051):
        assert not L.orc_is_prime(m), m
    for m in ((1 << 61) - 1, (1 << 31) - 1, 1000000007, 998244353):
        assert L.orc_is_prime(m), m


@pytest.mark.parametrize("logn,bits", [(4, [30, 30, 31]), (13, [40, 40, 40, 60]), (16, [60, 50, 50, 60, 60])])
def test_prime_chain(logn, bits):
    n = 1 << logn
    p = ckks.Params(logn, bits[:-1], bits[-1:], 1)
    taken = []
    for b, q in zip(bits, p.mod):
        # independent search for the first untaken prime 2^b - j*2n + 1
        j = 1
        while True:
            c = (1 << b) - j * 2 * n + 1
            if py_is_prime(c) and c not in taken:
                break
            j += 1
        assert q == c
        taken.append(q)
        assert q % (2 * n) == 1 and q < (1 << b)
    for q, psi in zip(p.mod, p.psi):
        assert pow(psi, n, q) == q - 1 and pow(psi, 2 * n, q) == 1


def negacyclic_schoolbook(a, b, q):
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                out[k] += a[i] * b[j]
            else:
                out[k - n] -= a[i] * b[j]
    return [x % q for x in out]


@pytest.mark.parametrize("n", [8, 16, 32, 64])
def test_ntt_and_polymul(n):
    L = ckks.lib()
    rng = np.random.default_rng(n)
    for bits in (30, 50, 60):
        q = int(L.orc_find_prime(bits, n, None, 0))
        psi = int(L.orc_find_psi(q, n))
        a = [int(x) for x in rng.integers(0, q, n, dtype=np.uint64)]
        b = [int(x) for x in rng.integers(0, q, n, dtype=np.uint64)]
        A = np.array(a, dtype=np.uint64)
        L.orc_ntt(ckks.ptr(A), n, q, psi)
        # direct evaluation at psi^(2k+1)
        for k in range(n):
            r = pow(psi, 2 * k + 1, q)
            assert int(A[k]) == sum(a[t] * pow(r, t, q) for t in range(n)) % q
        L.orc_intt(ckks.ptr(A), n, q, psi)
        assert [int(x) for x in A] == a
        out = np.zeros(n, dtype=np.uint64)
        L.orc_polymul(ckks.ptr(np.array(a, dtype=np.uint64)), ckks.ptr(np.array(b, dtype=np.uint64)),
                      ckks.ptr(out), n, q, psi)
        assert [int(x) for x in out] == negacyclic_schoolbook(a, b, q)


def chacha_vectors():
    rows = []
    for line in open(os.path.join(GOLD, "chacha20_rfc8439.txt")):
        if line.startswith("#") or not line.strip():
            continue
        key, ctr, nonce, block = line.split()
        rows.append((bytes.fromhex(key), int(ctr), bytes.fromhex(nonce), bytes.fromhex(block)))
    return rows


def test_chacha20_rfc8439():
    L = ckks.lib()
    rows = chacha_vectors()
    assert len(rows) == 2
    for key, ctr, nonce, block in rows:
        k = np.frombuffer(key, dtype="<u4").astype(np.uint32).copy()
        nn = np.frombuffer(nonce, dtype="<u4").astype(np.uint32).copy()
        out = np.zeros(16, dtype=np.uint32)
        L.orc_chacha20_block(ckks.ptr(k, ckks.u32p), ctr, ckks.ptr(nn, ckks.u32p), ckks.ptr(out, ckks.u32p))
        assert out.astype("<u4").tobytes() == block


def test_stream_layout_matches_block_function():
    """Word w of stream (seed, purpose, index) is u64 w%8 of block w/8 with the
    key = seed LE || 0^24 and nonce = purpose LE || index LE."""
    L = ckks.lib()
    seed, purpose, index = 0x0123456789ABCDEF, 7, 0x1122334455667788
    w = np.zeros(40, dtype=np.uint64)
    L.orc_stream_u64(seed, purpose, index, 3, 40, ckks.ptr(w))
    key = np.zeros(8, dtype=np.uint32)
    key[0], key[1] = seed & 0xFFFFFFFF, seed >> 32
    nonce = np.array([purpose, index & 0xFFFFFFFF, index >> 32], dtype=np.uint32)
    ks = b""
    for blk in range(6):
        out = np.zeros(16, dtype=np.uint32)
        L.orc_chacha20_block(ckks.ptr(key, ckks.u32p), blk, ckks.ptr(nonce, ckks.u32p), ckks.ptr(out, ckks.u32p))
        ks += out.astype("<u4").tobytes()
    words = np.frombuffer(ks, dtype="<u8")
    assert (w == words[3:43]).all()


def test_samplers():
    L = ckks.lib()
    n = 1 << 16
    t = np.zeros(n, dtype=np.int64)
    L.orc_sample_ternary(5, 1, 0, n, ckks.ptr(t, ckks.i64p))
    w = np.zeros(n, dtype=np.uint64)
    L.orc_stream_u64(5, 1, 0, 0, n, ckks.ptr(w))
    assert (t == (w % 3).astype(np.int64) - 1).all()
    counts = np.bincount(t + 1)
    assert all(abs(c / n - 1 / 3) < 0.01 for c in counts)

    g = np.zeros(n, dtype=np.int64)
    L.orc_sample_gauss(9, 3, 4, n, 3.2, ckks.ptr(g, ckks.i64p))
    assert abs(g.mean()) < 0.05 and abs(g.std() - 3.2) < 0.05 and np.abs(g).max() <= 19
    # the cumulative table against an independent double-precision computation
    T = np.zeros(19, dtype=np.uint64)
    L.orc_gauss_table(3.2, ckks.ptr(T))
    wts = [1.0] + [2 * math.exp(-i * i / (2 * 3.2 * 3.2)) for i in range(1, 20)]
    tot = sum(wts)
    acc = 0.0
    for i in range(19):
        acc += wts[i]
        assert abs(int(T[i]) - acc / tot * 2.0 ** 63) < 2.0 ** 12
    # sign bit and magnitude from the same word
    L.orc_stream_u64(9, 3, 4, 0, n, ckks.ptr(w))
    mags = np.searchsorted(T, w >> np.uint64(1), side="right")
    exp = np.where(w & np.uint64(1), -mags, mags)
    assert (g == exp).all()

    p = ckks.Params(10, [40, 50], [60], 1)
    pidx = ckks.u32arr([0, 1, 2])
    u = np.zeros((3, p.n), dtype=np.uint64)
    L.orc_sample_uniform(p.cref, 11, 2, 0, ckks.ptr(pidx, ckks.u32p), 3, ckks.ptr(u))
    w2 = np.zeros(2 * 3 * p.n, dtype=np.uint64)
    L.orc_stream_u64(11, 2, 0, 0, len(w2), ckks.ptr(w2))
    for l in range(3):
        q = p.mod[l]
        for c in range(0, p.n, 97):
            word = 2 * (l * p.n + c)
            assert int(u[l, c]) == ((int(w2[word]) << 64) | int(w2[word + 1])) % q
        assert abs(float(u[l].mean()) / q - 0.5) < 0.03
