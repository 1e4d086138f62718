"""Pins of the oracle's modular arithmetic, prime and root search, ring product and transform.

Each check compares the C oracle with something other than itself: Python
integers, sympy's primality test, a published parameter set, closed forms of
the ring product, and the evaluation definition of the transform.
"""
import json
import os
import random

import numpy as np
import pytest
import sympy

from oracle import core, pyref

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_mulmod_edges_against_python_ints():
    qs = [(1 << 50) - 27, 1125899906826241, 1152921504606830593, (1 << 62) - 57, 12289]
    for q in qs:
        edges = {0, 1, 2, q - 1, q - 2, q // 2, q // 2 + 1}
        for k in range(1, 63):
            for v in ((1 << k) - 1, 1 << k, (1 << k) + 1):
                edges.add(v % q)
        edges = sorted(edges)
        for a in edges:
            for b in edges[:: max(1, len(edges) // 25)]:
                assert core.mulmod(a, b, q) == (a * b) % q
                assert core.lib().orc_addmod(a, b, q) == (a + b) % q
                assert core.lib().orc_submod(a, b, q) == (a - b) % q


def test_is_prime_matches_sympy():
    rnd = random.Random(5)
    cands = [3215031751, 2152302898747, 3474749660383, 341550071728321, 3825123056546413051,
             (1 << 61) - 1, (1 << 62) - 57, 561, 1105, 25326001]
    cands += [rnd.randrange(1 << 40, 1 << 62) | 1 for _ in range(300)]
    cands += list(range(2, 400))
    for n in cands:
        assert core.is_prime(n) == sympy.isprime(n), n


@pytest.mark.parametrize("N,bits,L", [(2048, 54, 2), (4096, 50, 2), (8192, 50, 3), (16384, 50, 4), (8192, 60, 3)])
def test_find_primes_are_the_largest(N, bits, L):
    qs = core.find_primes(N, bits, L)
    assert len(qs) == L and qs == sorted(qs, reverse=True)
    m = 2 * N
    for q in qs:
        assert q < (1 << bits) and q % m == 1 and sympy.isprime(q)
    # no prime with the congruence is skipped between 2^bits and the smallest chosen q
    c = ((1 << bits) - 1) // m * m + 1
    if c >= (1 << bits):
        c -= m
    found = []
    while c >= qs[-1]:
        if sympy.isprime(c):
            found.append(c)
        c -= m
    assert found == qs


@pytest.mark.parametrize("N,q", [(8, 17), (16, 97), (16, 7681), (32, 7681), (256, 7681), (512, 12289), (1024, 12289)])
def test_min_psi_equals_linear_scan(N, q):
    assert core.min_psi(N, q) == core.min_psi_scan(N, q)


def test_min_psi_published_root():
    cases = json.load(open(os.path.join(GOLD, "ntt_params.json")))["cases"]
    for c in cases:
        assert pow(c["psi"], c["N"], c["q"]) == c["q"] - 1
        assert core.min_psi(c["N"], c["q"]) == c["psi"]


@pytest.mark.parametrize("N,bits,L", [(2048, 54, 2), (8192, 50, 3), (16384, 50, 4)])
def test_min_psi_is_primitive_2n_root(N, bits, L):
    qs, psis = core.params(N, L, bits)
    for q, psi in zip(qs, psis):
        assert pow(psi, N, q) == q - 1
        assert pow(psi, 2 * N, q) == 1
        # every odd power is again a root of X^N + 1; none is smaller than psi (sampled)
        r = psi
        for k in range(1, 2 * N, 2):
            if k > 1:
                r = r * psi * psi % q
            assert r >= psi
            if k > 200:
                break


def _rand_poly(rnd, N, q):
    return np.array([rnd.randrange(q) for _ in range(N)], dtype=np.uint64)


@pytest.mark.parametrize("N,q", [(4, 17), (8, 97), (16, 7681), (64, 12289), (32, 1125899906826241)])
def test_schoolbook_matches_python_bigints(N, q):
    rnd = random.Random(N)
    for _ in range(3):
        a, b = _rand_poly(rnd, N, q), _rand_poly(rnd, N, q)
        assert core.negacyclic_mul(a, b, q).tolist() == pyref.negacyclic_mul(a.tolist(), b.tolist(), q)


def test_schoolbook_closed_forms():
    q, N = 1125899906826241, 256
    rnd = random.Random(1)
    a = _rand_poly(rnd, N, q)
    one = np.zeros(N, np.uint64)
    one[0] = 1
    assert np.array_equal(core.negacyclic_mul(a, one, q), a)
    for s in (1, 7, N - 1):
        xs = np.zeros(N, np.uint64)
        xs[s] = 1
        expect = [(int(a[(k - s) % N]) if k >= s else (-int(a[k - s + N])) % q) for k in range(N)]
        assert core.negacyclic_mul(a, xs, q).tolist() == expect
    half = np.zeros(N, np.uint64)
    half[N // 2] = 1
    minus_one = np.zeros(N, np.uint64)
    minus_one[0] = q - 1
    assert np.array_equal(core.negacyclic_mul(half, half, q), minus_one)
    for k in (0, 5, N - 1):
        b = _rand_poly(rnd, N, q)
        assert core.negacyclic_coeff(a, b, q, k) == int(core.negacyclic_mul(a, b, q)[k])


@pytest.mark.parametrize("N,q", [(8, 17), (16, 7681), (32, 7681), (64, 12289)])
def test_ntt_definition_matches_evaluation(N, q):
    psi = core.min_psi(N, q)
    rnd = random.Random(3)
    a = _rand_poly(rnd, N, q)
    assert core.ntt_direct(a, q, psi).tolist() == pyref.ntt_eval(a.tolist(), q, psi)


@pytest.mark.parametrize("N,q", [(16, 7681), (256, 7681), (512, 12289), (256, 1125899906826241)])
def test_fast_transform_equals_definition_and_inverts(N, q):
    psi = core.min_psi(N, q)
    rnd = random.Random(4)
    a = _rand_poly(rnd, N, q)
    A = core.ntt_direct(a, q, psi)
    assert np.array_equal(core.ntt_fast(a, q, psi), A)
    assert np.array_equal(core.intt_direct(A, q, psi), a)
    assert np.array_equal(core.intt_fast(A, q, psi), a)


def test_convolution_theorem_pins_order_and_product():
    # the slot-wise product of two transforms is the transform of the ring product
    for N, q in [(64, 12289), (1024, 12289), (512, 1125899906826241)]:
        psi = core.min_psi(N, q)
        rnd = random.Random(N)
        a, b = _rand_poly(rnd, N, q), _rand_poly(rnd, N, q)
        A, B = core.ntt_fast(a, q, psi), core.ntt_fast(b, q, psi)
        AB = np.array([int(x) * int(y) % q for x, y in zip(A, B)], dtype=np.uint64)
        assert np.array_equal(core.intt_fast(AB, q, psi), core.negacyclic_mul(a, b, q))


def test_fast_transform_full_size_roundtrip_and_spot_definition():
    N = 8192
    qs, psis = core.params(N, 1, 50)
    q, psi = qs[0], psis[0]
    rnd = np.random.Generator(np.random.PCG64(7))
    a = rnd.integers(0, q, size=N, dtype=np.uint64)
    A = core.ntt_fast(a, q, psi)
    assert np.array_equal(core.intt_fast(A, q, psi), a)
    for k in (0, 1, 4095, 8191, 1234):
        assert int(A[k]) == core.ntt_coeff(a, q, psi, k)


def test_csr_cpmul_methods_agree_and_coeff_matches():
    N, L = 64, 2
    q, psi = core.params(N, L, 50)
    g = np.random.Generator(np.random.PCG64(11))
    ct = np.stack([np.stack([g.integers(0, qi, size=N, dtype=np.uint64) for qi in q]) for _ in range(2 * 5)]).reshape(5, 2, L, N)
    pt = np.stack([np.stack([g.integers(0, qi, size=N, dtype=np.uint64) for qi in q]) for _ in range(4)])
    row = np.array([0, 3, 3, 7], np.int32)
    cti = np.array([0, 1, 4, 2, 2, 3, 0], np.int32)
    pti = np.array([1, 0, 3, 2, 1, 0, 3], np.int32)
    o0 = core.csr_cpmul(ct, pt, row, cti, pti, q, psi, method=0)
    o1 = core.csr_cpmul(ct, pt, row, cti, pti, q, psi, method=1)
    o2 = core.csr_cpmul(ct, pt, row, cti, pti, q, psi, method=2)
    assert np.array_equal(o0, o1)
    assert np.array_equal(o0, o2)
    assert not o0[1].any()                         # an output with no terms is zero
    # against Python big ints, term by term
    for o in range(3):
        for c in range(2):
            for i in range(L):
                acc = [0] * N
                for t in range(row[o], row[o + 1]):
                    p = pyref.negacyclic_mul(ct[cti[t], c, i].tolist(), pt[pti[t], i].tolist(), q[i])
                    acc = [(x + y) % q[i] for x, y in zip(acc, p)]
                assert o0[o, c, i].tolist() == acc
    for (o, c, i, k) in [(0, 0, 0, 0), (2, 1, 1, 63), (2, 0, 1, 17)]:
        assert core.csr_cpmul_coeff(ct, pt, row, cti, pti, q, o, c, i, k) == int(o0[o, c, i, k])


def test_crt_compose_roundtrip():
    q, _ = core.params(8192, 3, 50)
    Q = q[0] * q[1] * q[2]
    rnd = random.Random(9)
    for _ in range(200):
        x = rnd.randrange(Q)
        assert pyref.crt_compose([x % qi for qi in q], q) == x


def test_lift_is_signed_residue():
    q = [1125899906826241, 12289]
    v = np.array([-5, 0, 7, -128, 127])
    r = core.lift(v, q)
    assert r.shape == (2, 5)
    for i, qi in enumerate(q):
        assert r[i].tolist() == [int(x) % qi for x in v]
