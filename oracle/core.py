"""ctypes wrappers over the C oracle (``oracle.c``).

Test infrastructure only.  The shared object is compiled from ``oracle.c`` with
gcc on first use if it is missing (``oracle/build.py`` does the same on demand).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

u64p = ctypes.POINTER(ctypes.c_uint64)
i32p = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        U64, U32, I32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
        sig = {
            "orc_mulmod": (U64, [U64, U64, U64]),
            "orc_addmod": (U64, [U64, U64, U64]),
            "orc_submod": (U64, [U64, U64, U64]),
            "orc_powmod": (U64, [U64, U64, U64]),
            "orc_is_prime": (ctypes.c_int, [U64]),
            "orc_find_primes": (ctypes.c_int, [U32, U32, U32, u64p]),
            "orc_min_psi": (U64, [U32, U64]),
            "orc_min_psi_scan": (U64, [U32, U64]),
            "orc_negacyclic_mul": (None, [u64p, u64p, U32, U64, u64p]),
            "orc_negacyclic_coeff": (U64, [u64p, u64p, U32, U64, U32]),
            "orc_ntt_coeff": (U64, [u64p, U32, U64, U64, U32]),
            "orc_ntt_direct": (None, [u64p, U32, U64, U64, u64p]),
            "orc_intt_direct": (None, [u64p, U32, U64, U64, u64p]),
            "orc_ntt_fast": (None, [u64p, U32, U64, U64, u64p]),
            "orc_intt_fast": (None, [u64p, U32, U64, U64, u64p]),
            "orc_csr_cpmul": (None, [u64p, u64p, i32p, i32p, i32p, U32, U32, U32, u64p, u64p, u64p, ctypes.c_int]),
            "orc_csr_cpmul_cached": (None, [u64p, u64p, U32, U32, i32p, i32p, i32p, U32, U32, U32, u64p, u64p, u64p]),
            "orc_csr_cpmul_coeff": (U64, [u64p, u64p, i32p, i32p, i32p, U32, U32, u64p, U32, U32, U32, U32]),
            "orc_ntt_planes": (None, [u64p, U32, U32, U32, u64p, u64p, u64p, ctypes.c_int]),
            "orc_negacyclic_mul_planes": (None, [u64p, u64p, U32, U32, U32, u64p, u64p]),
            "orc_num_threads": (ctypes.c_int, []),
            "orc_philox4x64": (None, [u64p, u64p, u64p]),
            "orc_expand_c1": (None, [U64, U64, U64, u64p, U32, U32, u64p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(u64p)


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(i32p)


def mulmod(a, b, q):
    return lib().orc_mulmod(a, b, q)


def powmod(a, e, q):
    return lib().orc_powmod(a, e, q)


def is_prime(n):
    return bool(lib().orc_is_prime(n))


def find_primes(N, bits, L):
    """The L largest primes q < 2^bits with q = 1 (mod 2N), largest first."""
    out = np.zeros(L, dtype=np.uint64)
    n = lib().orc_find_primes(N, bits, L, out.ctypes.data_as(u64p))
    if n != L:
        raise ValueError("not enough primes")
    return [int(v) for v in out]


def min_psi(N, q):
    """Smallest x with x^N = -1 (mod q)."""
    return int(lib().orc_min_psi(N, q))


def min_psi_scan(N, q):
    """Same value by scanning x = 2, 3, ... (small q only)."""
    return int(lib().orc_min_psi_scan(N, q))


def params(N, L, bits):
    """Moduli and roots for a ring: (q list, psi list)."""
    q = find_primes(N, bits, L)
    return q, [min_psi(N, qi) for qi in q]


def negacyclic_mul(a, b, q):
    a, pa = _u64(a)
    b, pb = _u64(b)
    N = a.shape[-1]
    c = np.zeros(N, dtype=np.uint64)
    lib().orc_negacyclic_mul(pa, pb, N, q, c.ctypes.data_as(u64p))
    return c


def negacyclic_coeff(a, b, q, k):
    a, pa = _u64(a)
    b, pb = _u64(b)
    return int(lib().orc_negacyclic_coeff(pa, pb, a.shape[-1], q, k))


def ntt_direct(a, q, psi):
    a, pa = _u64(a)
    out = np.zeros_like(a)
    lib().orc_ntt_direct(pa, a.shape[-1], q, psi, out.ctypes.data_as(u64p))
    return out


def intt_direct(A, q, psi):
    A, pA = _u64(A)
    out = np.zeros_like(A)
    lib().orc_intt_direct(pA, A.shape[-1], q, psi, out.ctypes.data_as(u64p))
    return out


def ntt_coeff(a, q, psi, k):
    a, pa = _u64(a)
    return int(lib().orc_ntt_coeff(pa, a.shape[-1], q, psi, k))


def ntt_fast(a, q, psi):
    a, pa = _u64(a)
    out = np.zeros_like(a)
    lib().orc_ntt_fast(pa, a.shape[-1], q, psi, out.ctypes.data_as(u64p))
    return out


def intt_fast(A, q, psi):
    A, pA = _u64(A)
    out = np.zeros_like(A)
    lib().orc_intt_fast(pA, A.shape[-1], q, psi, out.ctypes.data_as(u64p))
    return out


def ntt_planes(x, q, psi, inverse=False):
    """Transform every plane of an [..., L, N] array; plane (.., i, :) uses q[i], psi[i]."""
    x = np.ascontiguousarray(x, dtype=np.uint64)
    L, N = x.shape[-2], x.shape[-1]
    n = x.size // (L * N)
    out = np.zeros_like(x)
    qa, pq = _u64(q)
    sa, ps = _u64(psi)
    lib().orc_ntt_planes(x.ctypes.data_as(u64p), n, N, L, pq, ps, out.ctypes.data_as(u64p), int(inverse))
    return out


def negacyclic_mul_planes(a, b, q):
    """Schoolbook ring product of matching [..., L, N] arrays."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    assert a.shape == b.shape
    L, N = a.shape[-2], a.shape[-1]
    out = np.zeros_like(a)
    qa, pq = _u64(q)
    lib().orc_negacyclic_mul_planes(a.ctypes.data_as(u64p), b.ctypes.data_as(u64p), a.size // (L * N), N, L, pq,
                                    out.ctypes.data_as(u64p))
    return out


def csr_cpmul(ct, pt, row, ct_idx, pt_idx, q, psi, method=1):
    """Term-list multiply-accumulate (see ``orc_csr_cpmul``).

    ct: [n_ct, 2, L, N], pt: [n_pt, L, N]; returns [n_out, 2, L, N].
    method 0 = schoolbook ring products, 1 = through the oracle's transform,
    2 = the same with every input transformed once and cached.
    """
    ct, pct = _u64(ct)
    pt, ppt = _u64(pt)
    row, prow = _i32(row)
    ci, pci = _i32(ct_idx)
    pi, ppi = _i32(pt_idx)
    L, N = ct.shape[-2], ct.shape[-1]
    n_out = len(row) - 1
    out = np.zeros((n_out, 2, L, N), dtype=np.uint64)
    qa, pq = _u64(q)
    sa, ps = _u64(psi)
    if method == 2:
        lib().orc_csr_cpmul_cached(pct, ppt, ct.shape[0], pt.shape[0], prow, pci, ppi, n_out, N, L, pq, ps,
                                   out.ctypes.data_as(u64p))
    else:
        lib().orc_csr_cpmul(pct, ppt, prow, pci, ppi, n_out, N, L, pq, ps, out.ctypes.data_as(u64p), method)
    return out


def csr_cpmul_coeff(ct, pt, row, ct_idx, pt_idx, q, o, c, i, k):
    ct, pct = _u64(ct)
    pt, ppt = _u64(pt)
    row, prow = _i32(row)
    ci, pci = _i32(ct_idx)
    pi, ppi = _i32(pt_idx)
    L, N = ct.shape[-2], ct.shape[-1]
    qa, pq = _u64(q)
    return int(lib().orc_csr_cpmul_coeff(pct, ppt, prow, pci, ppi, N, L, pq, o, c, i, k))


def lift(values, q):
    """Residues of signed integers: v mod q_i in [0, q_i) for each prime; [..., N] -> [..., L, N].

    The lift is the identity on the integer (a reading: -5 becomes q_i - 5).
    """
    v = np.asarray(values, dtype=np.int64)
    return np.stack([np.remainder(v, np.int64(int(qi))).astype(np.uint64) for qi in q], axis=-2)


def num_threads():
    return int(lib().orc_num_threads())


def philox4x64(counter, key):
    """Philox4x64-10 of a 4-word counter under a 2-word key -> 4 words (uint64)."""
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64(c.ctypes.data_as(u64p), k.ctypes.data_as(u64p), out.ctypes.data_as(u64p))
    return out


def expand_c1(seed, j, q, N):
    """Component 1 of ciphertext j regenerated from the 2-word seed: [L, N] residues."""
    qa = np.ascontiguousarray(q, dtype=np.uint64)
    out = np.zeros((len(q), N), dtype=np.uint64)
    lib().orc_expand_c1(int(seed[0]), int(seed[1]), int(j), qa.ctypes.data_as(u64p), len(q), N,
                        out.ctypes.data_as(u64p))
    return out
