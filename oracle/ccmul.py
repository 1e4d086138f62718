"""Ciphertext-ciphertext multiplication with relinearization: the server's
preprocessing step of Section 3.2 (CryptoTrain-P), [r_x r_w] from [r_x], [r_w].

Test infrastructure only.  The paper names the operation (CCMul, Section 2 and
Section 3.2) and runs it in SEAL's BFV without stating the algorithm; the
reading here is the BFV product of Fan and Vercauteren with relinearization
by RNS-digit key switching:

  tensor   a = (a0, a1), b = (b0, b1), every coefficient lifted to the centred
           integer in (-Q/2, Q/2]; over Z[X]/(X^N + 1)
               x0 = a0 b0,   x1 = a0 b1 + a1 b0,   x2 = a1 b1,
           each summed over the products of an output when several are
           accumulated (one rounding and one relinearization per output);
  scale    d_c = round(t x_c / Q) mod Q (nearest integer; Q is odd, no ties);
  relin    gadget g_j = (Q/q_j) [(Q/q_j)^-1]_{q_j} (so g_j = 1 mod q_j and 0 mod
           the other primes), key rlk_j = ([-(a_j s + e_j) + g_j s^2]_Q, a_j) for
           j < L with a_j uniform and e_j small (inputs), and with
           D_j = [d2]_{q_j} taken as an integer in [0, q_j):
               out = (d0 + sum_j D_j rlk_j0,  d1 + sum_j D_j rlk_j1)  mod Q.
           Then out0 + out1 s = d0 + d1 s + d2 s^2 - sum_j D_j e_j (mod Q).

The exact integer products are multi-modular: the oracle's own transform over
primes of its own whose product exceeds twice the largest |x_c|, recombined by
the CRT in Python integers.  The rounding is Python integer arithmetic.
"""
import numpy as np

from . import bfv, core


def _crt_basis(moduli):
    M = 1
    for m in moduli:
        M *= int(m)
    return M, [(M // int(m)) * pow(M // int(m), -1, int(m)) for m in moduli]


def centred(poly, q):
    """[L, N] residues -> list of N Python integers in (-Q/2, Q/2]."""
    Q, basis = _crt_basis(q)
    L, N = poly.shape
    out = []
    for k in range(N):
        v = sum(int(poly[i, k]) * basis[i] for i in range(L)) % Q
        out.append(v - Q if 2 * v > Q else v)
    return out


def residues(values, q):
    """Python integers -> [L, N] residues."""
    return np.array([[int(v) % int(qi) for v in values] for qi in q], dtype=np.uint64)


def _product_primes(N, bound):
    """Primes of the oracle's own for an exact product with |x| <= bound."""
    n = 1
    while True:
        ps = core.find_primes(N, 61, n)
        M = 1
        for p in ps:
            M *= p
        if M > 2 * bound + 1:
            return ps
        n += 1


def tensor(pairs, q, N_empty=0):
    """Exact x0, x1, x2 (lists of N integers) of the sum over (a, b) in pairs of a (x) b.

    pairs: list of (a [2, L, N], b [2, L, N]) residue arrays.  Modulo each
    product prime the sums are term-list products of the oracle's C path:
    output 0 = sum a (x) b0 = (sum a0 b0, sum a1 b0), output 1 = sum a (x) b1.
    An empty list is the empty sum, zero (N must then be given)."""
    if not pairs:
        return [[0] * N_empty for _ in range(3)]
    L, N = pairs[0][0].shape[1:]
    Q = bfv.modulus(q)
    n = len(pairs)
    bound = 2 * n * N * (Q // 2 + 1) ** 2
    ps = _product_primes(N, bound)
    psis = [core.min_psi(N, p) for p in ps]
    cts = np.zeros((n, 2, len(ps), N), dtype=np.uint64)
    pts = np.zeros((2 * n, len(ps), N), dtype=np.uint64)
    for j, (a, b) in enumerate(pairs):
        for c in range(2):
            cts[j, c] = residues(centred(a[c], q), ps)
            pts[2 * j + c] = residues(centred(b[c], q), ps)
    row = np.array([0, n, 2 * n], np.int32)
    a_idx = np.array(list(range(n)) * 2, np.int32)
    b_idx = np.array([2 * j for j in range(n)] + [2 * j + 1 for j in range(n)], np.int32)
    o = core.csr_cpmul(cts, pts, row, a_idx, b_idx, ps, psis, method=2).astype(object)   # [2, 2, K, N]
    pa = np.array(ps, dtype=object)[:, None]
    xs = [o[0, 0], (o[0, 1] + o[1, 0]) % pa, o[1, 1]]
    M, basis = _crt_basis(ps)
    out = []
    for x in xs:
        vals = []
        for k in range(N):
            v = sum(int(x[i, k]) * basis[i] for i in range(len(ps))) % M
            vals.append(v - M if 2 * v > M else v)
        out.append(vals)
    return out


def scale_round(x, Q, t):
    """round(t x / Q) for Python integers (nearest, Q odd so no ties)."""
    return [(2 * t * v + Q) // (2 * Q) for v in x]


def _ring_mul(x, y, q, psi):
    """Product of [L, N] residue arrays over every prime, through the oracle's transform."""
    X = core.ntt_planes(x, q, psi)
    Y = core.ntt_planes(y, q, psi)
    P = np.stack([np.array([int(u) * int(v) % int(q[i]) for u, v in zip(X[i], Y[i])], dtype=np.uint64)
                  for i in range(len(q))])
    return core.ntt_planes(P, q, psi, inverse=True)


def relin_key(s, a, e, q, psi):
    """rlk [L, 2, L, N]: rlk_j = ([-(a_j s + e_j) + g_j s^2]_Q, a_j) (coefficient domain).

    s [N] ternary, a [L(j), L(i), N] uniform residues, e [L(j), N] small integers."""
    L = len(q)
    N = len(s)
    s_res = core.lift(s, q)
    s2 = _ring_mul(s_res, s_res, q, psi)
    rlk = np.zeros((L, 2, L, N), dtype=np.uint64)
    for j in range(L):
        a_s = _ring_mul(np.ascontiguousarray(a[j], dtype=np.uint64), s_res, q, psi)
        e_res = core.lift(e[j], q)
        for i in range(L):
            qi = int(q[i])
            v = [(-int(x) - int(y)) % qi for x, y in zip(a_s[i], e_res[i])]
            if i == j:                                       # g_j = 1 mod q_j, 0 mod the others
                v = [(u + int(w)) % qi for u, w in zip(v, s2[i])]
            rlk[j, 0, i] = np.array(v, dtype=np.uint64)
            rlk[j, 1, i] = a[j][i]
    return rlk


def relinearize(d0, d1, d2, rlk, q, psi):
    """(d0, d1, d2) [L, N] residue arrays -> [2, L, N]: (d0, d1) + sum_j D_j rlk_j."""
    L, N = d0.shape
    D = np.stack([core.lift(d2[j].astype(np.int64), q) for j in range(L)])   # D_j reduced mod every prime
    ks = core.csr_cpmul(np.ascontiguousarray(rlk), D, np.array([0, L], np.int32), np.arange(L, dtype=np.int32),
                        np.arange(L, dtype=np.int32), q, psi, method=2)[0]
    qa = np.array([int(v) for v in q], dtype=object)[:, None]
    return ((np.stack([d0, d1]).astype(object) + ks.astype(object)) % qa).astype(np.uint64)


def ccmul_acc(a_cts, b_cts, row, a_idx, b_idx, rlk, q, psi, t):
    """Output o = Relin(round(t/Q * sum over terms k of o of a[a_idx[k]] (x) b[b_idx[k]])).

    a_cts [n_a, 2, L, N], b_cts [n_b, 2, L, N], rlk [L, 2, L, N] -> [n_out, 2, L, N]."""
    Q = bfv.modulus(q)
    outs = []
    for o in range(len(row) - 1):
        pairs = [(a_cts[a_idx[k]], b_cts[b_idx[k]]) for k in range(row[o], row[o + 1])]
        x = tensor(pairs, q, a_cts.shape[-1])
        d = [residues(scale_round(xc, Q, t), q) for xc in x]
        outs.append(relinearize(d[0], d[1], d[2], rlk, q, psi))
    return np.stack(outs)


def three_component(a, b, q, t):
    """The unrelinearized product (d0, d1, d2) [3, L, N] of one pair."""
    Q = bfv.modulus(q)
    return np.stack([residues(scale_round(xc, Q, t), q) for xc in tensor([(a, b)], q)])


def decrypt3(d, s, q, psi, t):
    """m = round(t [d0 + d1 s + d2 s^2]_Q / Q) mod t for a three-component ciphertext."""
    s_res = core.lift(s, q)
    s2 = _ring_mul(s_res, s_res, q, psi)
    ph = bfv.phase(np.stack([d[0], d[1]]), s, q, psi).astype(object)
    ph += _ring_mul(np.ascontiguousarray(d[2]), s2, q, psi).astype(object)
    qa = np.array([int(v) for v in q], dtype=object)[:, None]
    ph = (ph % qa)
    Q = bfv.modulus(q)
    vals = [v % Q for v in centred(ph.astype(np.uint64), q)]
    return np.array([((2 * t * v + Q) // (2 * Q)) % t for v in vals], dtype=np.int64)
