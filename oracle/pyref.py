"""Pure-Python big-integer reference for tiny rings (test infrastructure only).

Written independently of ``oracle.c`` so that the C oracle can be pinned to
something other than itself: Python integers never overflow and ``%`` is exact,
so every function here is the textbook definition with no word-size concerns.
"""


def negacyclic_mul(a, b, q):
    """Product in Z_q[X]/(X^N+1) via X^N = -1 (Section 2, ring A_{N,p})."""
    n = len(a)
    c = [0] * (2 * n)
    for i, ai in enumerate(a):
        for j, bj in enumerate(b):
            c[i + j] += int(ai) * int(bj)
    return [(c[k] - c[k + n]) % q for k in range(n)]


def poly_eval(a, x, q):
    return sum(int(c) * pow(x, j, q) for j, c in enumerate(a)) % q


def bitrev(v, logn):
    return int(format(v, "0%db" % logn)[::-1], 2) if logn else 0


def ntt_eval(a, q, psi):
    """Slot k holds a(psi^(2*brv(k)+1)): evaluation at the odd powers of psi."""
    n = len(a)
    logn = n.bit_length() - 1
    return [poly_eval(a, pow(psi, 2 * bitrev(k, logn) + 1, q), q) for k in range(n)]


def is_prime_trial(n):
    if n < 2:
        return False
    d = 2
    while d * d <= n:
        if n % d == 0:
            return False
        d += 1
    return True


def crt_compose(residues, moduli):
    """The unique x in [0, prod(moduli)) with x = r_i mod q_i."""
    Q = 1
    for m in moduli:
        Q *= m
    x = 0
    for r, m in zip(residues, moduli):
        Mi = Q // m
        x += int(r) * Mi * pow(Mi, -1, m)
    return x % Q
