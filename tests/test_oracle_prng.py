"""Oracle pins for the seeded ciphertext component c1 (Section 7, Discussion: the client
sends a seed instead of c1 and the server regenerates it).

The generator is Philox4x64-10; numpy ships an implementation of the same
published generator (numpy.random.Philox), which pins the oracle's: numpy's
bit generator emits the block of counter + 1 first (it steps the 256-bit
counter before each block).  The reduction to residues is pinned against
Python's exact big-integer arithmetic on numpy's words."""
import numpy as np
import pytest

from oracle import bfv, core

T = 65537
MASK256 = (1 << 256) - 1


def _words(x):
    return [(x >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]


def _numpy_block(counter, key):
    """The Philox4x64-10 block of `counter` (4 words) from numpy's generator."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(counter))
    start = _words((c - 1) & MASK256)           # numpy steps the counter before its first block
    bg = np.random.Philox(counter=np.array(start, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((5, 0, 0, 0), (0x0123456789ABCDEF, 0xFEDCBA9876543210)),
    ((2 ** 64 - 1, 7, 2, 0), (1, 2)),          # carry into the second word under numpy's step
    ((8191, 255, 3, 0), (2 ** 64 - 1, 2 ** 63)),
])
def test_philox_matches_numpy(counter, key):
    assert [int(v) for v in core.philox4x64(counter, key)] == _numpy_block(counter, key)


def test_expand_c1_is_the_wide_reduction_of_the_generator():
    q, _ = core.params(1024, 3, 50)
    seed = (0x1234, 0x5678)
    for j in (0, 3):
        got = core.expand_c1(seed, j, q, 1024)
        for i, qi in enumerate(q):
            for k in (0, 1, 2, 511, 1023):
                w = _numpy_block((k, j, i, 0), seed)
                assert int(got[i, k]) == ((w[0] << 64) | w[1]) % int(qi), (j, i, k)


def test_expand_c1_residues_are_canonical_and_spread():
    q, _ = core.params(4096, 2, 50)
    a = core.expand_c1((7, 9), 0, q, 4096)
    for i, qi in enumerate(q):
        v = a[i].astype(np.float64) / float(qi)
        assert (a[i] < np.uint64(qi)).all()
        assert abs(v.mean() - 0.5) < 0.02
        counts = np.histogram(v, bins=16, range=(0.0, 1.0))[0]
        chi2 = ((counts - 256.0) ** 2 / 256.0).sum()
        assert chi2 < 60.0                      # 15 degrees of freedom; p ~ 1e-7 at 60
    # other seeds and ciphertext indices give other components
    assert not np.array_equal(a, core.expand_c1((7, 10), 0, q, 4096))
    assert not np.array_equal(a, core.expand_c1((7, 9), 1, q, 4096))


def test_encryption_with_a_regenerated_c1_decrypts():
    N, L = 256, 3
    q, psi = core.params(N, L, 50)
    g = np.random.Generator(np.random.PCG64(61))
    s = g.integers(-1, 2, size=N)
    m = g.integers(0, T, size=N)
    e = np.clip(np.rint(g.normal(0, 3.2, size=N)), -19, 19).astype(np.int64)
    a = core.expand_c1((11, 12), 5, q, N)
    ct = bfv.encrypt(m, s, a, e, q, psi, T)
    assert np.array_equal(ct[1], a)
    assert np.array_equal(bfv.decrypt(ct, s, q, psi, T), m)


def test_ternary_map_splits_the_words_in_thirds():
    third = (1 << 64) // 3                      # 2^64 = 3 * third + 1
    assert bfv.ternary_from_word(0) == -1
    assert bfv.ternary_from_word(third) == -1   # 3 * third < 2^64
    assert bfv.ternary_from_word(third + 1) == 0
    assert bfv.ternary_from_word(2 * third) == 0      # 3 * 2 * third = 2^65 - 2
    assert bfv.ternary_from_word(2 * third + 1) == 1  # 3 * (2 * third + 1) = 2^65 + 1
    assert bfv.ternary_from_word((1 << 64) - 1) == 1


def test_keygen_is_numpy_philox_mapped_to_ternary():
    sk = bfv.keygen(0xC0FFEE, 64)
    for k in (0, 1, 17, 63):
        w = _numpy_block((k, 0, 0, (1 << 64) - 1), (0xC0FFEE, 0))[0]
        assert int(sk[k]) == bfv.ternary_from_word(w)
    big = bfv.keygen(12345, 3000)
    assert set(np.unique(big).tolist()) <= {-1, 0, 1}
    counts = np.array([(big == v).sum() for v in (-1, 0, 1)])
    assert (np.abs(counts - 1000) < 130).all()   # about 4.5 sigma of a binomial(3000, 1/3)
    assert not np.array_equal(bfv.keygen(1, 64), bfv.keygen(2, 64))
