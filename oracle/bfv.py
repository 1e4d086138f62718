"""Test-only BFV-style encryption over an RNS modulus Q = q_0 ... q_{L-1}.

Test infrastructure only.  The paper encrypts with a public key (Section 2,
"HE") and states no parameters; the reading used here is secret-key
encryption, which decrypts identically and matches the threat model (only the
client holds the secret key):
    c1 = a                                   (a uniform per prime, given)
    c0 = -a*s + e + Delta*m   (mod q_i)      Delta = floor(Q / t)
    m  = round(t * [c0 + c1*s]_Q / Q) mod t
All randomness (s ternary, a uniform, e small) is an input.  Ring products go
through the C oracle; the CRT and the rounding use Python integers.
"""
import numpy as np

from . import core


def modulus(q):
    Q = 1
    for qi in q:
        Q *= int(qi)
    return Q


def encrypt(m, s, a, e, q, psi, t, method=1):
    """m[N] in [0,t), s[N] in {-1,0,1}, a[L,N] residues, e[N] ints -> ct[2, L, N]."""
    L, N = a.shape
    Q = modulus(q)
    delta = Q // t
    s_res = core.lift(s, q)
    a = np.ascontiguousarray(a, dtype=np.uint64)
    if method == 1:
        a_hat = core.ntt_planes(a, q, psi)
        s_hat = core.ntt_planes(s_res, q, psi)
        as_hat = np.zeros_like(a_hat)
        for i in range(L):
            as_hat[i] = _pointwise(a_hat[i], s_hat[i], q[i])
        a_s = core.ntt_planes(as_hat, q, psi, inverse=True)
    else:
        a_s = core.negacyclic_mul_planes(a, s_res, q)
    e_res = core.lift(e, q)
    ct = np.zeros((2, L, N), dtype=np.uint64)
    m = np.asarray(m, dtype=np.int64)
    for i in range(L):
        qi = int(q[i])
        dm = (np.array([(delta % qi) * int(v) % qi for v in m], dtype=object))
        c0 = [(-int(x) + int(y) + int(z)) % qi for x, y, z in zip(a_s[i], e_res[i], dm)]
        ct[0, i] = np.array(c0, dtype=np.uint64)
        ct[1, i] = a[i]
    return ct


def _pointwise(x, y, qi):
    return np.array([int(u) * int(v) % int(qi) for u, v in zip(x, y)], dtype=np.uint64)


def phase(ct, s, q, psi, method=1):
    """c0 + c1*s mod q_i, per prime -> [L, N]."""
    _, L, N = ct.shape
    s_res = core.lift(s, q)
    if method == 1:
        c1_hat = core.ntt_planes(ct[1], q, psi)
        s_hat = core.ntt_planes(s_res, q, psi)
        prod_hat = np.stack([_pointwise(c1_hat[i], s_hat[i], q[i]) for i in range(L)])
        prod = core.ntt_planes(prod_hat, q, psi, inverse=True)
    else:
        prod = core.negacyclic_mul_planes(np.ascontiguousarray(ct[1]), s_res, q)
    out = np.zeros((L, N), dtype=np.uint64)
    for i in range(L):
        qi = int(q[i])
        out[i] = np.array([(int(u) + int(v)) % qi for u, v in zip(ct[0, i], prod[i])], dtype=np.uint64)
    return out


def decrypt(ct, s, q, psi, t, method=1, coeffs=None):
    """Exact decryption -> m[N] in [0, t) (or only the listed coefficients)."""
    x = phase(ct, s, q, psi, method)
    Q = modulus(q)
    Qi = [Q // int(qi) for qi in q]
    Qi_inv = [pow(Qi[i], -1, int(q[i])) for i in range(len(q))]
    idx = range(x.shape[1]) if coeffs is None else coeffs
    out = []
    for k in idx:
        v = 0
        for i in range(len(q)):
            v += (int(x[i, k]) * Qi_inv[i] % int(q[i])) * Qi[i]
        v %= Q
        out.append(((2 * t * v + Q) // (2 * Q)) % t)
    return np.array(out, dtype=np.int64)


def noise_bits(ct, s, m, q, psi, t):
    """log2 of the largest |[c0 + c1 s - Delta m]_Q| (centred), for noise-budget checks."""
    x = phase(ct, s, q, psi)
    Q = modulus(q)
    delta = Q // t
    Qi = [Q // int(qi) for qi in q]
    Qi_inv = [pow(Qi[i], -1, int(q[i])) for i in range(len(q))]
    worst = 0
    for k in range(x.shape[1]):
        v = sum((int(x[i, k]) * Qi_inv[i] % int(q[i])) * Qi[i] for i in range(len(q))) % Q
        r = (v - delta * int(m[k])) % Q
        if r > Q // 2:
            r -= Q
        worst = max(worst, abs(r))
    return worst.bit_length()


def ternary_from_word(w):
    """A 64-bit word to {-1, 0, 1}: floor(3 w / 2^64) - 1 (the three thirds of
    [0, 2^64), each within one word of 2^64 / 3)."""
    return (3 * int(w) >> 64) - 1


def keygen(seed, N):
    """Ternary secret key from a 64-bit seed: sk[k] = ternary_from_word(w), w the
    first word of the Philox4x64-10 block of counter (k, 0, 0, 2^64 - 1) under
    key (seed, 0).  The generator is the published one (pinned to numpy's); the
    map to {-1, 0, 1} is the key generator's stated definition."""
    out = np.empty(N, dtype=np.int8)
    for k in range(N):
        out[k] = ternary_from_word(core.philox4x64([k, 0, 0, (1 << 64) - 1], [seed, 0])[0])
    return out
