"""Pins of the oracle's packings (Section 3.3) and of the test-only encryption.

Packings are checked against the paper's toy example and against scipy's
2-D correlation (a library routine) and direct integer sums on random tiny
shapes; the encryption against decryption, the homomorphic property of
Section 2 ("HE") and a noise bound.
"""
import json
import os

import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import bfv, core, packing, plain, pyref

GOLD = os.path.join(os.path.dirname(__file__), "golden")
T = 65537


def _ring_mul_int(a, b, N):
    """Integer (not modular) negacyclic product of int64 polynomials, exact via Python ints."""
    c = [0] * N
    nz_a = [(i, int(v)) for i, v in enumerate(a) if v]
    nz_b = [(j, int(v)) for j, v in enumerate(b) if v]
    for i, x in nz_a:
        for j, y in nz_b:
            k = i + j
            if k < N:
                c[k] += x * y
            else:
                c[k - N] -= x * y
    return np.array(c, dtype=object)


def _padded_degrees(H, W, h, P):
    """Row-major encoding of the zero-padded input (the prior scheme the toy example compares to)."""
    Wp = W + 2 * P
    deg_x = (P + H - 1) * Wp + (P + W - 1)
    deg_w = (h - 1) * Wp + (h - 1)
    return deg_x, deg_w


def test_toy_example_degrees_and_use():
    g0 = json.load(open(os.path.join(GOLD, "toy_example.json")))
    H, W, h, P = g0["H"], g0["W"], g0["h"], g0["P"]
    assert _padded_degrees(H, W, h, P) == (g0["padded_degree_input"], g0["padded_degree_kernel"])
    g = packing.ConvGeometry(1, H, W, h, P, 16)
    x = np.array([[1, 2], [3, 4]])
    w = np.array([[5, 6], [7, 8]])
    xh, wh = packing.pi_x(x, g.O, 16), packing.pi_w(w, g.O, 16)
    assert max(np.nonzero(xh)[0]) == g0["corr_degree_input"]
    assert max(np.nonzero(wh)[0]) == g0["corr_degree_kernel"]
    prod = _ring_mul_int(xh, wh, 16)
    used = [k for k in range(16) if prod[k] != 0]
    assert len(used) == g0["product_coefficients_used"] == g.span + 1
    out = packing.conv_extract(prod.astype(np.int64), g)
    assert list(out.shape) == g0["output_shape"]
    assert np.array_equal(out, plain.conv2d(x[None], w[None, None], P)[0])
    # every one of the 9 product coefficients is an output value (100% use)
    assert sorted(out.reshape(-1).tolist()) == sorted(int(v) for v in prod[:9])


def test_single_channel_equals_scipy_correlation():
    rnd = np.random.Generator(np.random.PCG64(21))
    for _ in range(40):
        H, W = rnd.integers(1, 7, size=2)
        h = int(rnd.integers(1, min(H, W) + 1))
        x = rnd.integers(-9, 10, size=(H, W))
        w = rnd.integers(-9, 10, size=(h, h))
        g = packing.ConvGeometry(1, H, W, h, 0, 256)
        prod = _ring_mul_int(packing.pi_x(x, g.O, 256), packing.pi_w(w, g.O, 256), 256)
        full = correlate2d(x, w, mode="full")          # (H+h-1) x (W+h-1)
        for u in range(H + h - 1):
            for v in range(W + h - 1):
                assert prod[u * g.O + v] == full[u, v]


def test_fit_condition_is_exact():
    # span + 1 coefficients fit; one fewer wraps around and changes a coefficient
    H, W, h = 5, 4, 3
    rnd = np.random.Generator(np.random.PCG64(2))
    x = rnd.integers(1, 9, size=(H, W))
    w = rnd.integers(1, 9, size=(h, h))
    g = packing.ConvGeometry(1, H, W, h, 1, 1024)
    full = correlate2d(x, w, mode="full")
    ok = _ring_mul_int(packing.pi_x(x, g.O, g.S), packing.pi_w(w, g.O, g.S), g.S)
    assert ok[g.span] == full[H + h - 2, W + h - 2]
    bad = _ring_mul_int(packing.pi_x(x, g.O, g.S - 1), packing.pi_w(w, g.O, g.S - 1), g.S - 1)
    assert bad[0] != full[0, 0]


@pytest.mark.parametrize("seed", range(8))
def test_multichannel_conv_equals_plain(seed):
    rnd = np.random.Generator(np.random.PCG64(100 + seed))
    C, M = int(rnd.integers(1, 5)), int(rnd.integers(1, 4))
    H, W = int(rnd.integers(2, 7)), int(rnd.integers(2, 7))
    h = int(rnd.integers(1, min(H, W, 3) + 1))
    P = int(rnd.integers(0, h))
    N = 128
    g = packing.ConvGeometry(C, H, W, h, P, N)
    x = rnd.integers(-128, 128, size=(C, H, W))
    w = rnd.integers(-128, 128, size=(M, C, h, h))
    xin = packing.pack_conv_input(x, g)
    wk = packing.pack_conv_weight(w, g)
    ref = plain.conv2d(x, w, P)
    for m in range(M):
        acc = np.zeros(N, dtype=object)
        for k in range(g.cb):
            acc = acc + _ring_mul_int(xin[k], wk[m, k], N)
        assert np.array_equal(packing.conv_extract(acc.astype(np.int64), g), ref[m])


def test_cifar_conv_geometry_matches_hand_count():
    # 3x32x32 input, 3x3 kernel, pad 1, N = 8192: O = 34, span = 33*34 + 33
    g = packing.ConvGeometry(3, 32, 32, 3, 1, 8192)
    assert (g.O, g.span, g.S, g.Cw, g.cb, g.Hout) == (34, 33 * 34 + 33, 1156, 7, 1, 32)


@pytest.mark.parametrize("seed", range(4))
def test_weight_gradient_packing_equals_plain(seed):
    rnd = np.random.Generator(np.random.PCG64(300 + seed))
    C, M = int(rnd.integers(1, 4)), int(rnd.integers(1, 3))
    H = W = int(rnd.integers(3, 6))
    h, P = 3, 1
    N = 512
    x = rnd.integers(-20, 20, size=(C, H, W))
    dy = rnd.integers(-20, 20, size=(M, H, W))       # same padding: Hout = H
    g = packing.dw_geometry(C, H, W, H, P, N)
    xin = packing.pack_conv_input(x, g)
    ref = plain.conv2d_weight_grad(x, dy, P, h)
    for m in range(M):
        dyp = packing.pi_w(dy[m], g.O, N)
        for k in range(g.cb):
            prod = _ring_mul_int(xin[k], dyp, N).astype(np.int64)
            c0, c1 = k * g.Cw, min(C, (k + 1) * g.Cw)
            got = np.zeros((c1 - c0, h, h), dtype=np.int64)
            for c in range(c0, c1):
                for a in range(h):
                    for b in range(h):
                        got[c - c0, a, b] = prod[(c - c0) * g.S + (a - P + H - 1) * g.O + (b - P + H - 1)]
            assert np.array_equal(got, ref[m, c0:c1])


def test_weight_gradient_geometry_16x16():
    g = packing.dw_geometry(16, 16, 16, 16, 1, 8192)
    assert (g.O, g.S, g.Cw, g.cb) == (31, 961, 8, 2)


@pytest.mark.parametrize("n_in,n_out,N", [(7, 3, 32), (20, 9, 64), (256, 10, 4096), (64, 40, 256)])
def test_fc_packing_equals_matvec(n_in, n_out, N):
    rnd = np.random.Generator(np.random.PCG64(n_in * n_out))
    g = packing.FcGeometry(n_in, n_out, N)
    assert (g.n_ow + 1) * g.n_iw - 1 <= N
    x = rnd.integers(-128, 128, size=n_in)
    Wm = rnd.integers(-128, 128, size=(n_out, n_in))
    xin = packing.pack_fc_input(x, g)
    wk = packing.pack_fc_weight(Wm, g)
    outs = np.zeros((g.out_ct, N), dtype=np.int64)
    for o in range(g.out_ct):
        acc = np.zeros(N, dtype=object)
        for j in range(g.in_ct):
            acc = acc + _ring_mul_int(xin[j], wk[o, j], N)
        outs[o] = acc.astype(np.int64)
    assert np.array_equal(packing.fc_extract(outs, g), plain.matvec(Wm, x))


def test_fc_plan_is_minimal_by_brute_force():
    for n_in, n_out, N in [(1024, 256, 8192), (1024, 256, 4096), (256, 10, 16384), (1024, 256, 16384)]:
        g = packing.FcGeometry(n_in, n_out, N)
        best = min(-(-n_in // a) * -(-n_out // b) for a in range(1, n_in + 1) for b in range(1, n_out + 1)
                   if (b + 1) * a - 1 <= N)
        assert g.n_cpmul == best


def test_complexity_identity_section_3_3():
    # N1 - N2 = floor((h+1)/2) H + floor((h-1)/2) h, as printed
    for H in range(1, 70):
        for h in range(1, 12):
            d = packing.cheetah_degree_full_padding(H, h) - packing.corr_degree_full_padding(H, h)
            assert d == (h + 1) // 2 * H + (h - 1) // 2 * h


def test_term_lists_shapes():
    row, cti, pti = packing.conv_terms(2, 3, 2)
    assert len(row) == 7 and row[-1] == 12
    row, cti, pti = packing.dw_terms(4, 3, 2)
    assert len(row) == 7 and row[-1] == 3 * 2 * 4 * 2
    row, cti, pti = packing.fc_terms(1, 11, 3)
    assert row[-1] == 33


# ---------------------------------------------------------------- encryption

def _keys(N, L, bits, seed):
    q, psi = core.params(N, L, bits)
    g = np.random.Generator(np.random.PCG64(seed))
    s = g.integers(-1, 2, size=N)
    return q, psi, g, s


def _enc(m, s, q, psi, g, N):
    a = np.stack([g.integers(0, qi, size=N, dtype=np.uint64) for qi in q])
    e = np.clip(np.rint(g.normal(0, 3.2, size=N)), -19, 19).astype(np.int64)
    return bfv.encrypt(m, s, a, e, q, psi, T)


@pytest.mark.parametrize("N,L,bits", [(64, 2, 50), (1024, 3, 50), (256, 3, 60)])
def test_decrypt_inverts_encrypt(N, L, bits):
    q, psi, g, s = _keys(N, L, bits, N + L)
    m = g.integers(0, T, size=N)
    ct = _enc(m, s, q, psi, g, N)
    assert np.array_equal(bfv.decrypt(ct, s, q, psi, T), m)
    assert np.array_equal(bfv.decrypt(ct, s, q, psi, T, method=0), m)


def test_encrypt_schoolbook_and_transform_agree():
    N = 64
    q, psi, g, s = _keys(N, 2, 50, 5)
    m = g.integers(0, T, size=N)
    a = np.stack([g.integers(0, qi, size=N, dtype=np.uint64) for qi in q])
    e = g.integers(-19, 20, size=N)
    assert np.array_equal(bfv.encrypt(m, s, a, e, q, psi, T, method=0), bfv.encrypt(m, s, a, e, q, psi, T, method=1))


def test_homomorphic_cpmul_accumulate():
    # Section 2 ("HE"): decrypting a sum of ciphertext x plaintext products gives the
    # plaintext sum of ring products mod t.
    N, L = 128, 3
    q, psi, g, s = _keys(N, L, 50, 77)
    K = 5
    ms = [g.integers(0, T, size=N) for _ in range(K)]
    ps = [g.integers(-128, 128, size=N) for _ in range(K)]
    cts = np.stack([_enc(m, s, q, psi, g, N) for m in ms])
    pts = np.stack([core.lift(p, q) for p in ps])
    row = np.array([0, K], np.int32)
    acc = core.csr_cpmul(cts, pts, row, np.arange(K, dtype=np.int32), np.arange(K, dtype=np.int32), q, psi)
    expect = [0] * N
    for m, p in zip(ms, ps):
        prod = pyref.negacyclic_mul(m.tolist(), [int(v) % T for v in p], T)
        expect = [(x + y) % T for x, y in zip(expect, prod)]
    assert bfv.decrypt(acc[0], s, q, psi, T).tolist() == expect


def test_noise_stays_far_below_delta():
    N, L = 256, 3
    q, psi, g, s = _keys(N, L, 50, 8)
    m = g.integers(0, T, size=N)
    ct = _enc(m, s, q, psi, g, N)
    assert bfv.noise_bits(ct, s, m, q, psi, T) <= 6           # |e| <= 19 plus rounding
    Q = bfv.modulus(q)
    assert (Q // T).bit_length() > 120
