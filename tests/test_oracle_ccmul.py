"""Oracle pins for the ciphertext-ciphertext product with relinearization
(Section 3.2, CryptoTrain-P preprocessing: the server forms [r_x r_w] from
[r_x] and [r_w]), CPU only.

- the exact tensor product and the rounding against a schoolbook product over
  the integers and exact rational rounding on a tiny ring;
- the three-component product decrypts (with 1, s, s^2) to the ring product of
  the messages mod t; the relinearized product decrypts the same, with its
  noise inside the budget, also at the benchmark ring N = 8192, L = 3;
- the relinearization key satisfies rlk_j0 + rlk_j1 s = g_j s^2 - e_j by
  brute-force ring products, and the gadget recomposes d2;
- accumulated products decrypt to the sum of the message products;
- a mask product made this way completes the online protocol: Dec(c) - p = x w.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

from oracle import bfv, ccmul, core, packing, plain, pyref

T = 65537


def _keys(N, L, bits, seed):
    q, psi = core.params(N, L, bits)
    g = np.random.Generator(np.random.PCG64(seed))
    return q, psi, g, g.integers(-1, 2, size=N)


def _enc(m, s, q, psi, g, N, t=T):
    a = np.stack([g.integers(0, qi, size=N, dtype=np.uint64) for qi in q])
    e = np.clip(np.rint(g.normal(0, 3.2, size=N)), -19, 19).astype(np.int64)
    return bfv.encrypt(np.remainder(m, t), s, a, e, q, psi, t)


def _rlk(s, q, psi, g):
    L, N = len(q), len(s)
    a = np.stack([np.stack([g.integers(0, qi, size=N, dtype=np.uint64) for qi in q]) for _ in range(L)])
    e = np.clip(np.rint(g.normal(0, 3.2, size=(L, N))), -19, 19).astype(np.int64)
    return ccmul.relin_key(s, a, e, q, psi), a, e


def _int_negacyclic(a, b):
    N = len(a)
    out = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            if k < N:
                out[k] += a[i] * b[j]
            else:
                out[k - N] -= a[i] * b[j]
    return out


def test_tensor_and_rounding_match_brute_force_on_a_tiny_ring():
    N, L, t = 8, 2, 257
    q, psi = core.params(N, L, 20)
    Q = q[0] * q[1]
    g = np.random.Generator(np.random.PCG64(70))
    pairs = [(np.stack([np.stack([g.integers(0, qi, size=N, dtype=np.uint64) for qi in q]) for _ in range(2)]),
              np.stack([np.stack([g.integers(0, qi, size=N, dtype=np.uint64) for qi in q]) for _ in range(2)]))
             for _ in range(3)]

    def lift(poly):                                   # the integer of the residues, centred
        vals = []
        for k in range(N):
            v = pyref.crt_compose([int(poly[i, k]) for i in range(L)], q)
            vals.append(v - Q if 2 * v > Q else v)
        return vals

    x = [[0] * N for _ in range(3)]
    for a, b in pairs:
        a0, a1, b0, b1 = lift(a[0]), lift(a[1]), lift(b[0]), lift(b[1])
        for slot, prods in ((0, [(a0, b0)]), (1, [(a0, b1), (a1, b0)]), (2, [(a1, b1)])):
            for u, v in prods:
                x[slot] = [p + r for p, r in zip(x[slot], _int_negacyclic(u, v))]
    got = ccmul.tensor(pairs, q)
    assert got == x
    for slot in range(3):
        want = [math.floor(Fraction(t * v, Q) + Fraction(1, 2)) for v in x[slot]]
        assert ccmul.scale_round(got[slot], Q, t) == want


@pytest.mark.parametrize("N,L,bits", [(1024, 3, 50), (2048, 2, 50), (512, 4, 60)])
def test_product_decrypts_to_the_ring_product(N, L, bits):
    q, psi, g, s = _keys(N, L, bits, 71 + N)
    ma, mb = g.integers(0, T, size=N), g.integers(0, T, size=N)
    ma[:3] = [0, 1, T - 1]
    A, B = _enc(ma, s, q, psi, g, N), _enc(mb, s, q, psi, g, N)
    want = core.negacyclic_mul(ma, mb, T).astype(np.int64)
    d = ccmul.three_component(A, B, q, T)
    assert np.array_equal(ccmul.decrypt3(d, s, q, psi, T), want)
    rlk, _, _ = _rlk(s, q, psi, g)
    out = ccmul.relinearize(d[0], d[1], d[2], rlk, q, psi)
    assert np.array_equal(bfv.decrypt(out, s, q, psi, T), want)
    Q = bfv.modulus(q)
    assert bfv.noise_bits(out, s, want, q, psi, T) < (Q // (2 * T)).bit_length() - 20


def test_relin_key_identity_and_gadget_by_brute_force():
    N, L = 32, 3
    q, psi, g, s = _keys(N, L, 50, 72)
    rlk, a, e = _rlk(s, q, psi, g)
    s_l = [int(v) for v in s]
    s2 = _int_negacyclic(s_l, s_l)
    for j in range(L):
        for i in range(L):
            qi = q[i]
            lhs = [(int(u) + v) % qi for u, v in zip(rlk[j, 0, i], pyref.negacyclic_mul([int(v) for v in rlk[j, 1, i]],
                                                                                        [v % qi for v in s_l], qi))]
            rhs = [((s2[k] if i == j else 0) - int(e[j, k])) % qi for k in range(N)]
            assert lhs == rhs, (j, i)
    # the gadget: sum_j [d]_{q_j} g_j = d (mod Q) for residues d
    Q = bfv.modulus(q)
    d = [int(v) for v in g.integers(0, 2 ** 62, size=5)]
    gj = [(Q // qj) * pow(Q // qj, -1, qj) for qj in q]
    for v in d:
        assert sum((v % qj) * gj[j] for j, qj in enumerate(q)) % Q == v % Q


def test_accumulated_products_decrypt_to_the_sum():
    N, L = 1024, 3
    q, psi, g, s = _keys(N, L, 50, 73)
    rlk, _, _ = _rlk(s, q, psi, g)
    ms = [g.integers(0, T, size=N) for _ in range(5)]
    cts = np.stack([_enc(m, s, q, psi, g, N) for m in ms])
    row, ai, bi = [0, 3, 4], [0, 1, 2, 3], [4, 4, 0, 3]         # out0 = m0 m4 + m1 m4 + m2 m0; out1 = m3^2
    out = ccmul.ccmul_acc(cts, cts, row, ai, bi, rlk, q, psi, T)
    for o in range(2):
        want = np.zeros(N, dtype=np.int64)
        for k in range(row[o], row[o + 1]):
            want = (want + core.negacyclic_mul(ms[ai[k]], ms[bi[k]], T).astype(np.int64)) % T
        assert np.array_equal(bfv.decrypt(out[o], s, q, psi, T), want), o


def test_mask_product_completes_the_online_protocol():
    # preprocessing: [r_x r_w] = CCMul([r_x], [r_w]) summed over the output's
    # terms; online: c = [x] (x) (w - r_w) + [w] (x) (x - r_x) + [r_x r_w]
    N, L, B, C, M, H, h, P = 256, 3, 2, 2, 2, 5, 3, 1
    q, psi, g, s = _keys(N, L, 50, 74)
    rlk, _, _ = _rlk(s, q, psi, g)
    geo = packing.ConvGeometry(C, H, H, h, P, N)
    x = g.integers(-128, 128, size=(B, C, H, H))
    w = g.integers(-128, 128, size=(M, C, h, h))
    xh = np.remainder(np.concatenate([packing.pack_conv_input(x[b], geo) for b in range(B)]), T)
    wh = np.remainder(packing.pack_conv_weight(w, geo).reshape(-1, N), T)
    rx, rw = g.integers(0, T, size=xh.shape), g.integers(0, T, size=wh.shape)
    row, cti, pti = packing.conv_terms(B, M, geo.cb)
    ct_rx = np.stack([_enc(p, s, q, psi, g, N) for p in rx])
    ct_rw = np.stack([_enc(p, s, q, psi, g, N) for p in rw])
    rr = ccmul.ccmul_acc(ct_rx, ct_rw, row, cti, pti, rlk, q, psi, T)
    ct_x = np.stack([_enc(p, s, q, psi, g, N) for p in xh])
    ct_w = np.stack([_enc(p, s, q, psi, g, N) for p in wh])
    xm, wm = np.remainder(xh - rx, T), np.remainder(wh - rw, T)
    t1 = core.csr_cpmul(ct_x, core.lift(wm, q), row, cti, pti, q, psi)
    t2 = core.csr_cpmul(ct_w, core.lift(xm, q), row, pti, cti, q, psi)
    qa = np.array(q, dtype=object)[None, :, None]
    for b in range(B):
        for m in range(M):
            o = b * M + m
            c = ((t1[o].astype(object) + t2[o].astype(object) + rr[o].astype(object)) % qa).astype(np.uint64)
            p = np.zeros(N, dtype=np.int64)
            for k in range(row[o], row[o + 1]):
                p = (p + core.negacyclic_mul(xm[cti[k]], wm[pti[k]], T).astype(np.int64)) % T
            d = (bfv.decrypt(c, s, q, psi, T) - p) % T
            assert np.array_equal(packing.conv_extract(d, geo), plain.mod_t(plain.conv2d(x[b], w[m:m + 1], P)[0], T))


@pytest.mark.parametrize("bits", [48, 50])
def test_noise_at_the_benchmark_ring(bits):
    # the benchmark ring with the default primes below 2^48, and with 50-bit primes
    N, L = 8192, 3
    q, psi, g, s = _keys(N, L, bits, 75)
    rlk, _, _ = _rlk(s, q, psi, g)
    ma, mb = g.integers(0, T, size=N), g.integers(0, T, size=N)
    A, B = _enc(ma, s, q, psi, g, N), _enc(mb, s, q, psi, g, N)
    out = ccmul.ccmul_acc(A[None], B[None], [0, 1], [0], [0], rlk, q, psi, T)[0]
    want = core.negacyclic_mul(ma, mb, T).astype(np.int64)
    assert np.array_equal(bfv.decrypt(out, s, q, psi, T), want)
    Q = bfv.modulus(q)
    assert bfv.noise_bits(out, s, want, q, psi, T) < (Q // (2 * T)).bit_length() - 40


def test_an_output_without_terms_is_the_zero_ciphertext():
    # the empty sum: no tensor, d = 0, and relinearizing zero digits adds nothing
    N, L = 256, 2
    q, psi, g, s = _keys(N, L, 50, 76)
    rlk, _, _ = _rlk(s, q, psi, g)
    cts = np.stack([_enc(g.integers(0, T, size=N), s, q, psi, g, N) for _ in range(2)])
    out = ccmul.ccmul_acc(cts, cts, [0, 1, 1], [0], [1], rlk, q, psi, T)
    assert not out[1].any()
    assert not bfv.decrypt(out[1], s, q, psi, T).any()
