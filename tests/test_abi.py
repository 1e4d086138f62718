"""The C-ABI library loads and exports every symbol that include/he.h declares (no GPU needed)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2409_16675_amd", "libhe.so")
HDR = os.path.join(ROOT, "include", "he.h")


def declared():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"^(?:he_status|const char \*)\s*(he_\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("he_ctx_create", "he_ntt_fwd", "he_ntt_inv", "he_cpmul_acc", "he_corr_conv2d", "he_encrypt",
              "he_decrypt", "he_plan_create", "he_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_2409_16675_amd import he
    missing = [n for n in declared() if n not in he.EXPORTED]
    assert not missing, missing


def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.he_status_str.restype = ctypes.c_char_p
    assert lib.he_status_str(0) == b"ok"
    assert lib.he_status_str(-3).startswith(b"out of memory")


def test_invalid_params_rejected_without_gpu():
    from paper_2409_16675_amd import he
    import pytest
    for kw in (dict(N=1000, L=2), dict(N=8192, L=0), dict(N=8192, L=3, t=1), dict(N=32768, L=2),
               dict(N=8192, L=3, prime_bits=60, arith=he.HE_ARITH_F64)):
        with pytest.raises(he.HeError) as ei:
            he.he_ctx_create(**kw)
        assert ei.value.status in (he.HE_EINVAL, he.HE_EUNSUPPORTED)
