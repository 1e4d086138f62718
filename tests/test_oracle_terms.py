"""Pins of the oracle's term lists: each list is run through the oracle's
schoolbook ring products (core.csr_cpmul, method 0, modulo one 50-bit prime)
and the extracted result is compared with a plaintext reference that uses no
term list at all.  Inputs are small signed integers, so every ring product is
an exact integer far below q/2 and its residue gives it back.

  * conv_terms: the batched multi-block conv (Section 3.3 with channel blocks);
  * dw_terms: the CryptoTrain-P weight-gradient pairing of Section 3.2,
    [X](dY - r_dY) + [dY](X - r_X), whose plaintext product and mask product
    (computed here with a pure-Python ring product, per (b, m, k)) turn the
    output into sum_b X_b dY_b, extracted by dw_extract and compared with the
    plaintext weight gradient; with r = 0 the output is twice that gradient;
  * fc_terms: FC chunking over several input and output polynomials;
  * WindowGeometry.terms: tiled inputs (Section 3.3 windows), overlap-added.

A mis-paired index in any of these generators changes an output, because
every input polynomial is drawn independently.
"""
import numpy as np
import pytest

from oracle import core, packing, plain

T = 65537


def _prime(N):
    q, psi = core.params(N, 1, 50)
    return q, psi


def _ring_mul_int(a, b, N):
    """Exact negacyclic product of integer polynomials (Python ints)."""
    c = [0] * N
    nz_b = [(j, int(v)) for j, v in enumerate(b) if v]
    for i, x in enumerate(a):
        x = int(x)
        if not x:
            continue
        for j, y in nz_b:
            k = i + j
            if k < N:
                c[k] += x * y
            else:
                c[k - N] -= x * y
    return np.array(c, dtype=object)


def _as_ct(polys, q):
    """Integer polynomials [n, N] -> ciphertext residues [n, 2, 1, N]; component 1
    carries 3x component 0, so both components go through the term lists."""
    polys = np.asarray(polys, dtype=np.int64)
    c0 = core.lift(polys, q)                          # [n, 1, N]
    c1 = core.lift(3 * polys, q)
    return np.stack([c0, c1], axis=1)


def _as_pt(polys, q):
    return core.lift(np.asarray(polys, dtype=np.int64), q)   # [n, 1, N]


def _signed(res, q):
    """Residues of one prime -> the integers in (-q/2, q/2] they stand for."""
    v = np.asarray(res, dtype=np.uint64).astype(object)
    qq = int(q)
    return np.array([int(x) - qq if int(x) > qq // 2 else int(x) for x in v.reshape(-1)], dtype=object).reshape(v.shape)


def _run(ct, pt, terms, q, psi):
    row, cti, pti = terms
    out = core.csr_cpmul(ct, pt, row, cti, pti, q, psi, method=0)
    c0 = _signed(out[:, 0, 0], q[0])
    c1 = _signed(out[:, 1, 0], q[0])
    assert all(int(a) * 3 == int(b) for a, b in zip(c0.reshape(-1), c1.reshape(-1))), "component 1 mismatch"
    return c0


@pytest.mark.parametrize("B,C,M,H,h,P,N", [(3, 5, 2, 4, 3, 1, 64), (2, 2, 3, 5, 3, 0, 128)])
def test_conv_terms_batched_blocks(B, C, M, H, h, P, N):
    rnd = np.random.Generator(np.random.PCG64(B * 100 + C))
    q, psi = _prime(N)
    g = packing.ConvGeometry(C, H, H, h, P, N)
    assert g.cb > 1 or B > 1
    x = rnd.integers(-9, 10, size=(B, C, H, H))
    w = rnd.integers(-9, 10, size=(M, C, h, h))
    ct = _as_ct(np.concatenate([packing.pack_conv_input(x[b], g) for b in range(B)]), q)
    pt = _as_pt(packing.pack_conv_weight(w, g).reshape(-1, N), q)
    out = _run(ct, pt, packing.conv_terms(B, M, g.cb), q, psi)
    for b in range(B):
        ref = plain.conv2d(x[b], w, P)
        for m in range(M):
            got = packing.conv_extract(out[b * M + m].astype(np.int64), g)
            assert np.array_equal(got, ref[m]), (b, m)


def _dw_case(seed, B, C, M, H, P, N, masked):
    rnd = np.random.Generator(np.random.PCG64(seed))
    q, psi = _prime(N)
    Ho = H                                           # h = 3, P = 1: same padding
    g = packing.dw_geometry(C, H, H, Ho, P, N)
    X = rnd.integers(-8, 9, size=(B, C, H, H))
    dY = rnd.integers(-8, 9, size=(B, M, Ho, Ho))
    Xp = np.stack([packing.pack_conv_input(X[b], g) for b in range(B)])           # [B, cb, N]
    Dp = np.stack([[packing.pi_w(dY[b, m], g.O, N) for m in range(M)] for b in range(B)])   # [B, M, N]
    if masked:
        rX = rnd.integers(0, T, size=(B, g.cb, N))   # masks uniform mod t over all coefficients
        rD = rnd.integers(0, T, size=(B, M, N))
    else:
        rX = np.zeros((B, g.cb, N), dtype=np.int64)
        rD = np.zeros((B, M, N), dtype=np.int64)
    # ciphertext layout [B][cb + M]: X blocks, then dY per output channel;
    # plaintext layout [B][M + cb]: dY - r_dY per output channel, then X - r_X blocks
    ct = _as_ct(np.concatenate([np.concatenate([Xp[b], Dp[b]]) for b in range(B)]), q)
    pt = _as_pt(np.concatenate([np.concatenate([Dp[b] - rD[b], Xp[b] - rX[b]]) for b in range(B)]), q)
    out = _run(ct, pt, packing.dw_terms(B, M, g.cb), q, psi)          # [M * cb, N]
    ref = sum(plain.conv2d_weight_grad(X[b], dY[b], P, 3) for b in range(B))
    return g, X, dY, Xp, Dp, rX, rD, out, ref


@pytest.mark.parametrize("B,C,M,H,N", [(3, 3, 2, 5, 128), (2, 4, 3, 4, 64), (1, 2, 2, 5, 256)])
def test_dw_terms_unmasked_give_twice_the_gradient(B, C, M, H, N):
    g, *_, out, ref = _dw_case(400 + B, B, C, M, H, 1, N, masked=False)
    assert g.cb > 1 or N == 256
    polys = np.array([[int(v) for v in o] for o in out], dtype=object).reshape(M, g.cb, N)
    got = packing.dw_extract(polys, g)
    assert np.array_equal(got.astype(object), (2 * ref).astype(object))


@pytest.mark.parametrize("B,C,M,H,N", [(3, 3, 2, 5, 128), (2, 4, 3, 4, 64)])
def test_dw_terms_masked_protocol_identity(B, C, M, H, N):
    # Section 3.2: Dec(c) - p + [r_x r_w] = x w, per output polynomial and summed over b
    g, X, dY, Xp, Dp, rX, rD, out, ref = _dw_case(500 + B, B, C, M, H, 1, N, masked=True)
    assert g.cb > 1
    polys = np.zeros((M, g.cb, N), dtype=object)
    for m in range(M):
        for k in range(g.cb):
            acc = out[m * g.cb + k].copy()
            for b in range(B):
                acc = acc - _ring_mul_int(Xp[b, k] - rX[b, k], Dp[b, m] - rD[b, m], N)
                acc = acc + _ring_mul_int(rX[b, k], rD[b, m], N)
            polys[m, k] = acc
    got = packing.dw_extract(polys, g)
    assert np.array_equal(got.astype(object), ref.astype(object))


def test_dw_extract_reads_the_documented_coefficients():
    # a single channel product laid out by hand: dW[m, c, a, b] sits at
    # (c % Cw) * S + (a - P + h' - 1) * O + (b - P + h' - 1) of block c // Cw
    g = packing.dw_geometry(3, 4, 4, 4, 1, 64)
    polys = np.arange(2 * g.cb * 64, dtype=np.int64).reshape(2, g.cb, 64)
    got = packing.dw_extract(polys, g)
    assert got.shape == (2, 3, 3, 3)
    for m in range(2):
        for c in range(3):
            for a in range(3):
                for b in range(3):
                    k, cc = divmod(c, g.Cw)
                    assert got[m, c, a, b] == polys[m, k, cc * g.S + (a + 2) * g.O + (b + 2)]


@pytest.mark.parametrize("B,n_in,n_out,N", [(2, 20, 20, 32), (3, 30, 7, 64)])
def test_fc_terms_several_chunks(B, n_in, n_out, N):
    rnd = np.random.Generator(np.random.PCG64(n_in * 7 + B))
    q, psi = _prime(N)
    g = packing.FcGeometry(n_in, n_out, N)
    assert g.in_ct > 1
    x = rnd.integers(-20, 21, size=(B, n_in))
    Wm = rnd.integers(-20, 21, size=(n_out, n_in))
    ct = _as_ct(np.concatenate([packing.pack_fc_input(x[b], g) for b in range(B)]), q)
    pt = _as_pt(packing.pack_fc_weight(Wm, g).reshape(-1, N), q)
    out = _run(ct, pt, packing.fc_terms(B, g.in_ct, g.out_ct), q, psi)
    for b in range(B):
        got = packing.fc_extract(out[b * g.out_ct:(b + 1) * g.out_ct].astype(np.int64), g)
        assert np.array_equal(got, plain.matvec(Wm, x[b])), b


def test_fc_terms_more_than_one_output_polynomial():
    g = packing.FcGeometry(20, 20, 32)
    assert g.in_ct > 1 and g.out_ct > 1
    test_fc_terms_several_chunks(2, 20, 20, 32)


@pytest.mark.parametrize("B,C,M,H,W,h,P,N", [(2, 2, 2, 12, 10, 3, 1, 64), (1, 3, 2, 9, 9, 3, 0, 64)])
def test_window_terms_overlap_add(B, C, M, H, W, h, P, N):
    rnd = np.random.Generator(np.random.PCG64(H * W + C))
    q, psi = _prime(N)
    g = packing.WindowGeometry(C, M, H, W, h, P, N)
    assert g.tiles > 1
    x = rnd.integers(-9, 10, size=(B, C, H, W))
    w = rnd.integers(-9, 10, size=(M, C, h, h))
    ct = _as_ct(np.concatenate([g.pack_input(x[b]).reshape(-1, N) for b in range(B)]), q)
    pt = _as_pt(g.pack_weight(w).reshape(-1, N), q)
    out = _run(ct, pt, g.terms(B), q, psi)
    for b in range(B):
        ref = plain.conv2d(x[b], w, P)
        for m in range(M):
            polys = [out[(b * g.tiles + t) * M + m].astype(np.int64) for t in range(g.tiles)]
            assert np.array_equal(g.extract(polys), ref[m]), (b, m)
