"""Oracle pins for the online linear-layer protocol of Section 3.2 (CPU only).

The server holds [x], [w] and the precomputed [r_x r_w], plus the client's
masked plaintexts (x - r_x) and (w - r_w).  It returns
    c = [x] (x) (w - r_w) + [w] (x) (x - r_x) + [r_x r_w]      (2 CPMul + 2 CCAdd)
    p = (x - r_x)(w - r_w)                                      (PPMul, mod t)
and the client computes Dec(c) - p = x w.  The plaintext product mod t is the
oracle's ring product with q = t; it is pinned here against the pure-Python
product, and the whole identity against the plaintext convolution.
"""
import numpy as np
import pytest

from oracle import bfv, core, packing, plain, pyref

T = 65537


def test_ring_product_mod_t_matches_pure_python():
    # the plaintext product is the ring product of Section 2 over Z_t
    g = np.random.Generator(np.random.PCG64(11))
    for N in (16, 64):
        a = g.integers(0, T, size=N)
        b = g.integers(0, T, size=N)
        assert core.negacyclic_mul(a, b, T).tolist() == pyref.negacyclic_mul(a.tolist(), b.tolist(), T)


def test_t_admits_a_negacyclic_transform():
    # 65537 - 1 = 2^16, so 2N divides t - 1 for every N <= 2^15 and the minimal
    # root psi with psi^N = -1 exists; the transform's evaluation definition holds
    for N in (1024, 8192, 16384):
        psi = core.min_psi(N, T)
        assert pow(psi, N, T) == T - 1
    N = 64
    psi = core.min_psi(N, T)
    g = np.random.Generator(np.random.PCG64(12))
    a, b = g.integers(0, T, size=N), g.integers(0, T, size=N)
    A, B = core.ntt_direct(a, T, psi), core.ntt_direct(b, T, psi)
    prod = core.intt_direct(np.array([int(x) * int(y) % T for x, y in zip(A, B)], dtype=np.uint64), T, psi)
    assert prod.tolist() == pyref.negacyclic_mul(a.tolist(), b.tolist(), T)


def _keys(N, L, seed):
    q, psi = core.params(N, L, 50)
    g = np.random.Generator(np.random.PCG64(seed))
    s = g.integers(-1, 2, size=N)
    return q, psi, g, s


def _enc(m, s, q, psi, g, N):
    a = np.stack([g.integers(0, qi, size=N, dtype=np.uint64) for qi in q])
    e = np.clip(np.rint(g.normal(0, 3.2, size=N)), -19, 19).astype(np.int64)
    return bfv.encrypt(np.remainder(m, T), s, a, e, q, psi, T)


@pytest.mark.parametrize("B,C,M,H,h,P", [(2, 2, 2, 5, 3, 1), (1, 3, 2, 4, 3, 0)])
def test_online_protocol_recovers_the_convolution(B, C, M, H, h, P):
    N, L = 256, 3
    q, psi, g, s = _keys(N, L, 100 + B + C)
    geo = packing.ConvGeometry(C, H, H, h, P, N)
    x = g.integers(-128, 128, size=(B, C, H, H))
    w = g.integers(-128, 128, size=(M, C, h, h))
    xh = np.remainder(np.concatenate([packing.pack_conv_input(x[b], geo) for b in range(B)]), T)   # [B*cb, N]
    wh = np.remainder(packing.pack_conv_weight(w, geo).reshape(-1, N), T)                          # [M*cb, N]
    rx = g.integers(0, T, size=xh.shape)
    rw = g.integers(0, T, size=wh.shape)
    row, cti, pti = packing.conv_terms(B, M, geo.cb)
    n_out = len(row) - 1
    # client: ciphertexts of x, w and of the precomputed mask products
    ct_x = np.stack([_enc(p, s, q, psi, g, N) for p in xh])
    ct_w = np.stack([_enc(p, s, q, psi, g, N) for p in wh])
    rr = []
    for o in range(n_out):
        acc = [0] * N
        for k in range(row[o], row[o + 1]):
            pr = pyref.negacyclic_mul(rx[cti[k]].tolist(), rw[pti[k]].tolist(), T)
            acc = [(u + v) % T for u, v in zip(acc, pr)]
        rr.append(_enc(np.array(acc), s, q, psi, g, N))
    # server: two CPMul-accumulates (the second with the roles of the operands swapped) and the CCAdds
    xm = np.remainder(xh - rx, T)
    wm = np.remainder(wh - rw, T)
    t1 = core.csr_cpmul(ct_x, core.lift(wm, q), row, cti, pti, q, psi)
    t2 = core.csr_cpmul(ct_w, core.lift(xm, q), row, pti, cti, q, psi)
    qa = np.array(q, dtype=object)[None, :, None]
    c = np.stack([((t1[o].astype(object) + t2[o].astype(object) + rr[o].astype(object)) % qa).astype(np.uint64)
                  for o in range(n_out)])
    # server: the plaintext product of the masked operands
    p = []
    for o in range(n_out):
        acc = np.zeros(N, dtype=np.int64)
        for k in range(row[o], row[o + 1]):
            acc = (acc + core.negacyclic_mul(xm[cti[k]], wm[pti[k]], T).astype(np.int64)) % T
        p.append(acc)
    # client: Dec(c) - p = x (x) w, whose block-0 coefficients are the convolution
    for b in range(B):
        for m in range(M):
            o = b * M + m
            d = (bfv.decrypt(c[o], s, q, psi, T).astype(np.int64) - p[o]) % T
            got = packing.conv_extract(d, geo)
            ref = plain.mod_t(plain.conv2d(x[b], w[m:m + 1], P)[0], T)
            assert np.array_equal(got, ref), (b, m)
