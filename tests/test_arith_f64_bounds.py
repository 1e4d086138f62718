"""The fp64 modular arithmetic of the device (exact products through one FMA,
lazy reduction) on the CPU, instruction by instruction in IEEE double
precision: every product is congruent to the exact product mod q, and its
magnitude stays within the bounds the compile-time reduction planner and the
multiply-accumulate rely on (mul_out, mulv_out, the reduced bound 0.51 q and
the 31 q limit), at worst-case operands for primes just below 2^48; and the
store of the inverse transform's outputs (|x| < q, no reduction) yields the
canonical residue.

Python floats are IEEE binary64 with correctly rounded * and +, round() ties
to even like rint, and a fused multiply-add is formed exactly with rationals
and rounded once."""
import random
from fractions import Fraction

import pytest

from oracle import core

LIMIT, REDUCED = 31.0, 0.51


def mul_out(b):
    return 0.5 + 0.0625 * b + 0.01


def mulv_out(b):
    return 0.5 + 0.09375 * b + 0.01


def fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def rint(x):
    return float(round(x))


def mul(q, y, w, wq):
    h = y * w
    l = fma(y, w, -h)
    k = rint(y * wq)
    r = fma(-k, q, h)
    return r + l


def reduce(q, qinv, x):
    return fma(-rint(x * qinv), q, x)


def store_out(q, qinv, x):
    # floor(x / q) in {-1, 0} from one estimate, then q added back when negative
    t = rint(fma(x, qinv, -0.5))
    return fma(-t, q, x)


def operands(q, bound, rng, n):
    """Integers of magnitude up to bound * q: the extremes, and random ones."""
    top = int(bound * q)
    xs = [top, -top, top - 1, -(top - 1), q - 1, -(q - 1), 1, -1, 0]
    xs += [rng.randrange(-top, top + 1) for _ in range(n)]
    return [float(x) for x in xs]


PRIMES = [int(q) for q in core.find_primes(8192, 48, 3)] + [int(q) for q in core.find_primes(16384, 48, 2)]


@pytest.mark.parametrize("q", PRIMES)
def test_twiddle_product_exact_and_bounded(q):
    rng = random.Random(q)
    qf = float(q)
    assert q < 2 ** 48 and qf == q
    ws = [q - 1, q - 2, (q - 1) // 2, 1, 2] + [rng.randrange(q) for _ in range(20)]
    for b in (1.0, 4.0, 8.0, 16.0, 24.0, LIMIT):
        for y in operands(q, b, rng, 40):
            for w in ws:
                wq = float(Fraction(w, q))   # the table's fl(w / q)
                r = mul(qf, y, float(w), wq)
                assert r == int(r), (y, w)
                assert (int(r) - int(y) * w) % q == 0, (y, w)
                assert abs(r) <= mul_out(b) * q, (b, y, w, r / q)


@pytest.mark.parametrize("q", PRIMES)
def test_product_with_formed_companion_exact_and_bounded(q):
    # mulv: the companion fl(b * fl(1/q)) formed in the kernel; b a residue of
    # either sign (canonical, or a reduced double of the workspace), or a
    # twiddle taken without its companion by a transform pass, whose inputs
    # reach the 31 q limit
    rng = random.Random(q + 1)
    qf, qinv = float(q), 1.0 / float(q)
    bs = [q - 1, -(q - 1), int(REDUCED * q), -int(REDUCED * q), 1, -1] + [rng.randrange(-q + 1, q) for _ in range(20)]
    for b_in in (0.51, 1.0, 4.0, 8.0, 16.0, 24.0, LIMIT):
        for y in operands(q, b_in, rng, 40):
            for b in bs:
                r = mul(qf, y, float(b), float(b) * qinv)
                assert r == int(r)
                assert (int(r) - int(y) * b) % q == 0
                assert abs(r) <= mulv_out(b_in) * q, (b_in, y, b, r / q)


@pytest.mark.parametrize("q", PRIMES)
def test_reduce_and_accumulated_chunk(q):
    rng = random.Random(q + 2)
    qf, qinv = float(q), 1.0 / float(q)
    for x in operands(q, LIMIT, rng, 400):
        r = reduce(qf, qinv, x)
        assert r == int(r) and (int(r) - int(x)) % q == 0
        assert abs(r) <= REDUCED * q, (x, r / q)
    # the multiply-accumulate's worst chunk: a fold, then 48 products of canonical
    # operands at their bound, stays below the limit and exact
    worst = REDUCED * q + 48 * mulv_out(1.0) * q
    assert worst <= LIMIT * q < 2 ** 53
    acc = float(int(REDUCED * q))
    for _ in range(48):
        acc += mul(qf, float(q - 1), float(q - 1), float(q - 1) * qinv)
    assert acc == int(acc) and abs(acc) <= worst


@pytest.mark.parametrize("q", PRIMES)
def test_store_of_outputs_below_q(q):
    # the planner keeps the last stage's products below 0.99 q; every integer
    # |x| < q, the edges included, reaches its canonical residue exactly
    rng = random.Random(q + 3)
    qf, qinv = float(q), 1.0 / float(q)
    assert mul_out(0.48 / 0.0625) <= 0.99 + 1e-12 < 1.0
    h = q // 2
    xs = [0, 1, -1, 2, -2, q - 1, -(q - 1), q - 2, -(q - 2), h, -h, h + 1, -(h + 1), h - 1, -(h - 1)]
    xs += [rng.randrange(-q + 1, q) for _ in range(4000)]
    for x in xs:
        r = store_out(qf, qinv, float(x))
        assert r == int(r) and int(r) == x % q, (x, r)


def test_bounds_used_by_the_kernels_are_the_ones_checked():
    # the constants the device policy declares (arith.hpp) equal the ones above
    import os
    import re
    src = open(os.path.join(os.path.dirname(__file__), "..", "paper_2409_16675_amd", "csrc", "arith.hpp")).read()
    f64 = src[src.index("struct ArF64"):src.index("struct ArU64")]
    assert re.search(r"kLimit = 31\.0;", f64) and re.search(r"kReduced = 0\.51;", f64)
    assert "mul_out(double b_in) { return 0.5 + 0.0625 * b_in + 0.01; }" in f64
    assert "mulv_out(double b_in) { return 0.5 + 0.09375 * b_in + 0.01; }" in f64
    assert re.search(r"kStoreIn = 0\.99;", f64)
    body = f64[f64.index("uint64_t store_out(V x) const {"):]
    body = body[:body.index("}")]
    assert "__builtin_rint(__builtin_fma(x, qinv, -0.5))" in body and "__builtin_fma(-t, q, x)" in body
