"""Thin ctypes binding of libhe.so (C ABI in include/he.h), same names as the C calls.

Only argument marshalling happens here: device buffers are torch tensors (their
data pointers are passed through), streams are torch streams.  Every step of
the computation runs in the library's HIP kernels.  If libhe.so is missing the
import fails loudly: there is no fallback.
"""
import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# HE_LIBRARY selects another build of the same library (the host-sanitizer build)
LIB_PATH = os.environ.get("HE_LIBRARY") or os.path.join(_PKG, "libhe.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("%s is not built (run paper_2409_16675_amd.build.build() or __graft_entry__.build())" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)

HE_OK = 0
HE_EINVAL, HE_EUNSUPPORTED, HE_ENOMEM, HE_EDEVICE, HE_ERANGE, HE_EBUSY, HE_ETIMEOUT = -1, -2, -3, -4, -5, -6, -7
HE_ARITH_AUTO, HE_ARITH_F64, HE_ARITH_U64 = 0, 1, 2
HE_IN_NTT, HE_OUT_NTT, HE_ACCUMULATE, HE_VALIDATE, HE_PLAIN_POLY, HE_UNFUSED = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
HE_PACK_NONE, HE_PACK_FUSED, HE_PACK_MEMORY = 0, 1, 2
HE_IN_RESIDENT = 0x40
HE_KIND_CONV, HE_KIND_DW, HE_KIND_FC, HE_KIND_DX = 0, 1, 2, 3
HE_PREPARE_PPMUL, HE_PREPARE_CCMUL = 0x1, 0x2
HE_NOALLOC_SCRATCH_MB = 64
F64_MAX_BITS = 48          # HE_ARITH_F64 needs every prime below 2^48

c_void_p, c_u32, c_u64, c_i32, c_size = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_size_t
u64p = ctypes.POINTER(ctypes.c_uint64)
i32p = ctypes.POINTER(ctypes.c_int32)
i64p = ctypes.POINTER(ctypes.c_int64)


class he_params(ctypes.Structure):
    _fields_ = [("N", c_u32), ("L", c_u32), ("prime_bits", c_u32), ("arith", c_u32), ("q", u64p), ("t", c_u64),
                ("device", c_i32), ("reserved", c_i32)]


class he_conv_shape(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("B", c_u32), ("C", c_u32), ("M", c_u32), ("H", c_u32), ("W", c_u32), ("h", c_u32),
                ("P", c_u32), ("n_in", c_u32), ("n_out", c_u32), ("stride", c_u32)]


class he_plan_info(ctypes.Structure):
    _fields_ = [(n, c_i32 if n == "kind" else c_u32) for n in
                ("kind", "N", "O", "span", "S", "Cw", "cb", "Hout", "Wout", "n_iw", "n_ow", "n_ct_in", "n_pt",
                 "n_ct_out", "n_terms", "Hw", "Ww", "tiles")]


class he_layer_info(ctypes.Structure):
    _fields_ = [("workspace_bytes", c_u64), ("off_ct_hat", c_u64), ("off_pt_poly", c_u64), ("off_pt_hat", c_u64),
                ("off_acc", c_u64), ("off_flag", c_u64), ("fwd_ct_planes", c_u32), ("fwd_pt_planes", c_u32),
                ("mac_planes", c_u32), ("inv_planes", c_u32), ("pack", c_u32), ("reserved", c_u32)]


_SIGS = {
    "he_ctx_create": [ctypes.POINTER(he_params), ctypes.POINTER(c_void_p)],
    "he_ctx_destroy": [c_void_p],
    "he_ctx_moduli": [c_void_p, u64p, u64p],
    "he_ctx_info": [c_void_p, ctypes.POINTER(c_u32), ctypes.POINTER(c_u32), ctypes.POINTER(c_u64),
                    ctypes.POINTER(c_u32)],
    "he_ctx_set_schedule": [c_void_p, c_u32, c_u32, c_u32],
    "he_ctx_get_schedule": [c_void_p, c_u32, ctypes.POINTER(c_u32), ctypes.POINTER(c_u32)],
    "he_ctx_profile": [c_void_p, ctypes.c_int],
    "he_ctx_profile_read": [c_void_p, c_void_p, c_u32, ctypes.POINTER(c_u32)],
    "he_ntt_fwd": [c_void_p, c_void_p, c_u32, c_void_p],
    "he_ntt_inv": [c_void_p, c_void_p, c_u32, c_void_p],
    "he_cpmul_acc": [c_void_p, c_void_p, c_void_p, c_u32, c_void_p, c_u32, c_void_p, c_size, c_void_p],
    "he_cpmul_acc_ws": [c_void_p, c_u32, c_u32, ctypes.POINTER(c_size)],
    "he_plan_create": [c_void_p, ctypes.POINTER(he_conv_shape), ctypes.POINTER(c_void_p)],
    "he_plan_destroy": [c_void_p],
    "he_plan_get_info": [c_void_p, ctypes.POINTER(he_plan_info)],
    "he_plan_query": [c_u32, ctypes.POINTER(he_conv_shape), ctypes.POINTER(he_plan_info)],
    "he_plan_create_host": [c_u32, ctypes.POINTER(he_conv_shape), ctypes.POINTER(c_void_p)],
    "he_layer_query": [c_void_p, c_u32, c_u32, ctypes.POINTER(he_layer_info)],
    "he_ccmul_ws_size": [c_void_p, c_u32, c_u32, c_u32, c_u32, c_u32, ctypes.POINTER(c_size)],
    "he_ccmul": [c_void_p, c_void_p, c_u32, c_void_p, c_u32, i32p, i32p, i32p, c_u32, c_void_p, c_void_p, c_u32,
                 c_void_p, c_size, c_void_p],
    "he_plan_terms": [c_void_p, i32p, i32p, i32p],
    "he_workspace_size": [c_void_p, c_u32, ctypes.POINTER(c_size)],
    "he_corr_conv2d": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_u32, c_void_p, c_size, c_void_p],
    "he_corr_conv2d_noalloc": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_u32, c_void_p],
    "he_ppmul_ws_size": [c_void_p, c_u32, ctypes.POINTER(c_size)],
    "he_corr_conv2d_seeded": [c_void_p, c_void_p, c_void_p, u64p, c_void_p, c_void_p, c_u32, c_void_p, c_size,
                              c_void_p],
    "he_expand_c1": [c_void_p, u64p, c_u32, c_u32, c_void_p, c_void_p],
    "he_ppmul": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_u32, c_void_p, c_size, c_void_p],
    "he_ctx_prepare": [c_void_p, c_u32, c_u32, c_u32],
    "he_keygen": [c_void_p, c_u64, c_void_p],
    "he_pack_input": [c_void_p, i32p, i64p],
    "he_extract_output": [c_void_p, i64p, i64p],
    "he_encrypt": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
    "he_decrypt": [c_void_p, c_void_p, c_void_p, c_u32, i64p, c_void_p],
    "he_autotune": [c_void_p, c_u32, ctypes.c_char_p, c_void_p, c_void_p, c_u32, ctypes.POINTER(c_u32)],
    "he_batch_create": [c_i32, ctypes.POINTER(c_void_p)],
    "he_batch_add": [c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_u32)],
    "he_batch_build": [c_void_p, c_u32],
    "he_batch_rebind": [c_void_p, c_u32, c_void_p],
    "he_batch_run": [c_void_p, c_void_p],
    "he_batch_sync": [c_void_p, c_void_p],
    "he_batch_set_spin_limit": [c_void_p, c_u32],
    "he_batch_get_info": [c_void_p, c_void_p],
    "he_batch_destroy": [c_void_p],
    "he_server_create": [c_void_p, ctypes.POINTER(c_void_p)],
    "he_server_submit": [c_void_p, c_void_p, c_void_p, c_u64, c_u32, ctypes.POINTER(c_u64)],
    "he_server_wait": [c_void_p, c_u64, ctypes.c_int64, c_void_p],
    "he_server_drain": [c_void_p],
    "he_server_close_session": [c_void_p, c_u64],
    "he_server_replay": [c_void_p, c_u32, c_void_p, c_void_p, c_void_p, c_void_p, c_u32, c_void_p],
    "he_server_stats": [c_void_p, c_void_p],
    "he_server_destroy": [c_void_p],
}
for _n, _a in _SIGS.items():
    _f = getattr(_lib, _n)
    _f.argtypes = _a
    _f.restype = c_i32
_lib.he_status_str.argtypes = [c_i32]
_lib.he_status_str.restype = ctypes.c_char_p
_lib.he_last_error.argtypes = []
_lib.he_last_error.restype = ctypes.c_char_p

EXPORTED = sorted(list(_SIGS) + ["he_status_str", "he_last_error"])


class HeError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s: %s (%s)" % (where, _lib.he_status_str(status).decode(), _lib.he_last_error().decode()))


def _chk(st, where):
    if st != HE_OK:
        raise HeError(st, where)


def _stream(stream):
    if stream is None:
        return c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return c_void_p(stream)
    return c_void_p(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if t.numel() and not t.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return c_void_p(t.data_ptr())
    return c_void_p(t)


def lib():
    return _lib


# ------------------------------------------------------------------ contexts
def he_ctx_create(N, L, prime_bits=48, t=65537, q=None, arith=HE_ARITH_AUTO, device=0):
    p = he_params()
    p.N, p.L, p.prime_bits, p.arith, p.t, p.device = N, L, prime_bits, arith, t, device
    qa = None
    if q is not None:
        qa = (c_u64 * L)(*[int(v) for v in q])
        p.q = ctypes.cast(qa, u64p)
    h = c_void_p()
    _chk(_lib.he_ctx_create(ctypes.byref(p), ctypes.byref(h)), "he_ctx_create")
    return h


def he_ctx_destroy(ctx):
    _chk(_lib.he_ctx_destroy(ctx), "he_ctx_destroy")


def he_ctx_moduli(ctx, L):
    q = (c_u64 * L)()
    psi = (c_u64 * L)()
    _chk(_lib.he_ctx_moduli(ctx, ctypes.cast(q, u64p), ctypes.cast(psi, u64p)), "he_ctx_moduli")
    return [int(v) for v in q], [int(v) for v in psi]


def he_ctx_info(ctx):
    N, L, a = c_u32(), c_u32(), c_u32()
    t = c_u64()
    _chk(_lib.he_ctx_info(ctx, ctypes.byref(N), ctypes.byref(L), ctypes.byref(t), ctypes.byref(a)), "he_ctx_info")
    return N.value, L.value, t.value, a.value


HE_OP_FWD, HE_OP_INV, HE_OP_MAC = 0, 1, 2


def he_ctx_set_schedule(ctx, op, arith, loge):
    _chk(_lib.he_ctx_set_schedule(ctx, op, arith, loge), "he_ctx_set_schedule")


def he_ctx_get_schedule(ctx, op):
    a, le = c_u32(), c_u32()
    _chk(_lib.he_ctx_get_schedule(ctx, op, ctypes.byref(a), ctypes.byref(le)), "he_ctx_get_schedule")
    return a.value, le.value


def compiled_schedules(N, f64_ok=True):
    """(arith, loge) pairs compiled for ring degree N (mirrors the library's table)."""
    logn = N.bit_length() - 1
    out = []
    for a in (HE_ARITH_F64, HE_ARITH_U64):
        if a == HE_ARITH_F64 and not f64_ok:
            continue
        for le in (3, 4, 5):
            if 10 <= logn <= 14 and 6 <= logn - le <= 10:
                out.append((a, le))
    return out


class he_kernel_stat(ctypes.Structure):
    _fields_ = [("kind", c_u32), ("launches", c_u32), ("total_ms", ctypes.c_double), ("max_ms", ctypes.c_double)]


KERNEL_KINDS = {0: "ntt_fwd", 1: "ntt_fwd_lift", 2: "ntt_inv", 3: "mac_inv", 4: "mac", 5: "pack", 6: "persistent", 7: "rns_convert"}


def he_ctx_profile(ctx, enable):
    _chk(_lib.he_ctx_profile(ctx, 1 if enable else 0), "he_ctx_profile")


def he_ctx_profile_read(ctx):
    arr = (he_kernel_stat * 8)()
    n = c_u32()
    _chk(_lib.he_ctx_profile_read(ctx, ctypes.cast(arr, c_void_p), 8, ctypes.byref(n)), "he_ctx_profile_read")
    return {KERNEL_KINDS[arr[i].kind]: dict(launches=arr[i].launches, total_ms=arr[i].total_ms, max_ms=arr[i].max_ms)
            for i in range(n.value)}


def he_ntt_fwd(ctx, planes, n_polys, stream=None):
    _chk(_lib.he_ntt_fwd(ctx, _ptr(planes), n_polys, _stream(stream)), "he_ntt_fwd")


def he_ntt_inv(ctx, planes, n_polys, stream=None):
    _chk(_lib.he_ntt_inv(ctx, _ptr(planes), n_polys, _stream(stream)), "he_ntt_inv")


def he_cpmul_acc_ws(ctx, K, flags=0):
    b = c_size()
    _chk(_lib.he_cpmul_acc_ws(ctx, K, flags, ctypes.byref(b)), "he_cpmul_acc_ws")
    return b.value


def he_cpmul_acc(ctx, ct, pt, K, acc, flags=0, ws=None, ws_bytes=0, stream=None):
    _chk(_lib.he_cpmul_acc(ctx, _ptr(ct), _ptr(pt), K, _ptr(acc), flags, _ptr(ws), ws_bytes, _stream(stream)),
         "he_cpmul_acc")


# ------------------------------------------------------------------ plans
def he_plan_create(ctx, kind, B=1, C=0, M=0, H=0, W=0, h=0, P=0, n_in=0, n_out=0, stride=0):
    s = he_conv_shape(kind, B, C, M, H, W, h, P, n_in, n_out, stride)
    h_ = c_void_p()
    _chk(_lib.he_plan_create(ctx, ctypes.byref(s), ctypes.byref(h_)), "he_plan_create")
    return h_


def he_plan_destroy(plan):
    _chk(_lib.he_plan_destroy(plan), "he_plan_destroy")


def he_plan_get_info(plan):
    i = he_plan_info()
    _chk(_lib.he_plan_get_info(plan, ctypes.byref(i)), "he_plan_get_info")
    return {n: getattr(i, n) for n, _ in he_plan_info._fields_}


def he_plan_query(N, kind, B=1, C=0, M=0, H=0, W=0, h=0, P=0, n_in=0, n_out=0, stride=0):
    """Plan info for ring degree N without a context or device (host only)."""
    s = he_conv_shape(kind, B, C, M, H, W, h, P, n_in, n_out, stride)
    i = he_plan_info()
    _chk(_lib.he_plan_query(N, ctypes.byref(s), ctypes.byref(i)), "he_plan_query")
    return {n: getattr(i, n) for n, _ in he_plan_info._fields_}


def he_plan_create_host(N, kind, B=1, C=0, M=0, H=0, W=0, h=0, P=0, n_in=0, n_out=0, stride=0):
    """Client-side plan on ring degree N: no context, no device memory."""
    s = he_conv_shape(kind, B, C, M, H, W, h, P, n_in, n_out, stride)
    out = c_void_p()
    _chk(_lib.he_plan_create_host(N, ctypes.byref(s), ctypes.byref(out)), "he_plan_create_host")
    return out.value


def he_layer_query(plan, L=0, flags=0):
    """Host-only setup of one layer call: workspace regions, planes per stage, packing."""
    i = he_layer_info()
    _chk(_lib.he_layer_query(plan, L, flags, ctypes.byref(i)), "he_layer_query")
    return {n: getattr(i, n) for n, _ in he_layer_info._fields_ if n != "reserved"}


def he_plan_terms(plan):
    info = he_plan_get_info(plan)
    row = np.zeros(info["n_ct_out"] + 1, np.int32)
    cti = np.zeros(info["n_terms"], np.int32)
    pti = np.zeros(info["n_terms"], np.int32)
    _chk(_lib.he_plan_terms(plan, row.ctypes.data_as(i32p), cti.ctypes.data_as(i32p), pti.ctypes.data_as(i32p)),
         "he_plan_terms")
    return row, cti, pti


def he_workspace_size(plan, flags=0):
    b = c_size()
    _chk(_lib.he_workspace_size(plan, flags, ctypes.byref(b)), "he_workspace_size")
    return b.value


def he_corr_conv2d(ctx, plan, ct_in, plain, ct_out, flags=0, ws=None, ws_bytes=0, stream=None):
    _chk(_lib.he_corr_conv2d(ctx, plan, _ptr(ct_in), _ptr(plain), _ptr(ct_out), flags, _ptr(ws), ws_bytes,
                             _stream(stream)), "he_corr_conv2d")


def he_corr_conv2d_noalloc(ctx, plan, ct_in, plain, ct_out, flags=0, stream=None):
    """he_corr_conv2d with the library's fixed device scratch instead of a workspace (allocates nothing)."""
    _chk(_lib.he_corr_conv2d_noalloc(ctx, plan, _ptr(ct_in), _ptr(plain), _ptr(ct_out), flags, _stream(stream)),
         "he_corr_conv2d_noalloc")


def _seed(seed):
    s = np.ascontiguousarray(np.array([int(seed[0]), int(seed[1])], dtype=np.uint64))
    return s, s.ctypes.data_as(u64p)


def he_corr_conv2d_seeded(ctx, plan, ct0, seed, plain, ct_out, flags=0, ws=None, ws_bytes=0, stream=None):
    """he_corr_conv2d with input component 1 regenerated from `seed` (two 64-bit words); ct0 [n][L][N]."""
    keep, ps = _seed(seed)
    _chk(_lib.he_corr_conv2d_seeded(ctx, plan, _ptr(ct0), ps, _ptr(plain), _ptr(ct_out), flags, _ptr(ws), ws_bytes,
                                    _stream(stream)), "he_corr_conv2d_seeded")


def he_expand_c1(ctx, seed, first_ct, n_ct, out, stream=None):
    keep, ps = _seed(seed)
    _chk(_lib.he_expand_c1(ctx, ps, first_ct, n_ct, _ptr(out), _stream(stream)), "he_expand_c1")


def he_ctx_prepare(ctx, ops, ccmul_max_out=0, ccmul_max_terms=0):
    """Build the resources of he_ppmul / he_ccmul ahead of their calls (HE_PREPARE_* bits)."""
    _chk(_lib.he_ctx_prepare(ctx, ops, ccmul_max_out, ccmul_max_terms), "he_ctx_prepare")


def he_keygen(ctx, seed):
    """Ternary secret key [N] (int8, host) from a 64-bit seed."""
    N = he_ctx_info(ctx)[0]
    sk = np.zeros(N, dtype=np.int8)
    _chk(_lib.he_keygen(ctx, seed, sk.ctypes.data), "he_keygen")
    return sk


def he_ppmul_ws_size(plan, flags=0):
    b = c_size()
    _chk(_lib.he_ppmul_ws_size(plan, flags, ctypes.byref(b)), "he_ppmul_ws_size")
    return b.value


def he_ppmul(ctx, plan, a, b, out, flags=0, ws=None, ws_bytes=0, stream=None):
    """out[o] = sum over the plan's terms of a[cti] * b[pti] in Z_t[X]/(X^N+1) (device buffers)."""
    _chk(_lib.he_ppmul(ctx, plan, _ptr(a), _ptr(b), _ptr(out), flags, _ptr(ws), ws_bytes, _stream(stream)),
         "he_ppmul")


def he_ccmul_ws_size(ctx, n_a, n_b, n_out, n_terms, flags=0):
    b = c_size()
    _chk(_lib.he_ccmul_ws_size(ctx, n_a, n_b, n_out, n_terms, flags, ctypes.byref(b)), "he_ccmul_ws_size")
    return b.value


def he_ccmul(ctx, a, n_a, b, n_b, row, a_idx, b_idx, n_out, rlk_hat, out, flags=0, ws=None, ws_bytes=0, stream=None):
    """out[o] = Relin(round(t/Q * sum over terms of a[a_idx] (x) b[b_idx])) (device ciphertexts; host
    int32 term lists, row None for pairwise products)."""
    if row is None:
        rp = ap = bp = None
    else:
        row = np.ascontiguousarray(row, dtype=np.int32)
        a_idx = np.ascontiguousarray(a_idx, dtype=np.int32)
        b_idx = np.ascontiguousarray(b_idx, dtype=np.int32)
        rp, ap, bp = (v.ctypes.data_as(i32p) for v in (row, a_idx, b_idx))
    _chk(_lib.he_ccmul(ctx, _ptr(a), n_a, _ptr(b), n_b, rp, ap, bp, n_out, _ptr(rlk_hat), _ptr(out), flags, _ptr(ws),
                       ws_bytes, _stream(stream)), "he_ccmul")


def he_pack_input(plan, x, n_out_words):
    x = np.ascontiguousarray(x, dtype=np.int32)
    out = np.zeros(n_out_words, dtype=np.int64)
    _chk(_lib.he_pack_input(plan, x.ctypes.data_as(i32p), out.ctypes.data_as(i64p)), "he_pack_input")
    return out


def he_extract_output(plan, polys, n_out_values):
    polys = np.ascontiguousarray(polys, dtype=np.int64)
    y = np.zeros(n_out_values, dtype=np.int64)
    _chk(_lib.he_extract_output(plan, polys.ctypes.data_as(i64p), y.ctypes.data_as(i64p)), "he_extract_output")
    return y


# ------------------------------------------------------------------ encryption
def he_encrypt(ctx, s, m, a, e, ct, stream=None):
    _chk(_lib.he_encrypt(ctx, _ptr(s), _ptr(m), _ptr(a), _ptr(e), _ptr(ct), _stream(stream)), "he_encrypt")


def he_decrypt(ctx, s, ct, n_ct, N, stream=None):
    m = np.zeros(n_ct * N, dtype=np.int64)
    _chk(_lib.he_decrypt(ctx, _ptr(s), _ptr(ct), n_ct, m.ctypes.data_as(i64p), _stream(stream)), "he_decrypt")
    return m.reshape(n_ct, N)


# ------------------------------------------------------------------ autotuning
class he_tune_entry(ctypes.Structure):
    _fields_ = [("op", c_u32), ("arith", c_u32), ("loge", c_u32), ("exact", c_u32), ("us", ctypes.c_double)]


def he_autotune(ctx, n_polys=512, cache_path=None, stream=None):
    arr = (he_tune_entry * 64)()
    n = c_u32()
    _chk(_lib.he_autotune(ctx, n_polys, cache_path.encode() if cache_path else None, _stream(stream),
                          ctypes.cast(arr, c_void_p), 64, ctypes.byref(n)), "he_autotune")
    return [dict(op=arr[i].op, arith=arr[i].arith, loge=arr[i].loge, exact=bool(arr[i].exact), us=arr[i].us)
            for i in range(n.value)]


# ------------------------------------------------------------------ batching
HE_BATCH_GRAPH, HE_BATCH_STRICT_SYNC, HE_BATCH_PROFILE = 0x1, 0x2, 0x4


class he_job(ctypes.Structure):
    _fields_ = [("plan", c_void_p), ("ct_in", c_void_p), ("plain", c_void_p), ("ct_out", c_void_p), ("flags", c_u32),
                ("reserved", c_u32)]


class he_batch_info(ctypes.Structure):
    _fields_ = [("n_jobs", c_u32), ("n_tasks", c_u32), ("grid", c_u32), ("arith", c_u32), ("cpmul", c_u64),
                ("fwd_planes", c_u64), ("inv_planes", c_u64), ("ws_bytes", c_u64), ("kernel_launches", c_u64),
                ("kernel_ms", ctypes.c_double)]


def _job(plan, ct_in, plain, ct_out, flags):
    return he_job(plan.value if isinstance(plan, c_void_p) else plan, _ptr(ct_in).value, _ptr(plain).value,
                  _ptr(ct_out).value, flags, 0)


def he_batch_create(device=0):
    h = c_void_p()
    _chk(_lib.he_batch_create(device, ctypes.byref(h)), "he_batch_create")
    return h


def he_batch_add(b, ctx, plan, ct_in, plain, ct_out, flags=0):
    j = _job(plan, ct_in, plain, ct_out, flags)
    idx = c_u32()
    _chk(_lib.he_batch_add(b, ctx, ctypes.byref(j), ctypes.byref(idx)), "he_batch_add")
    return idx.value


def he_batch_build(b, flags=HE_BATCH_GRAPH):
    _chk(_lib.he_batch_build(b, flags), "he_batch_build")


def he_batch_rebind(b, index, plan, ct_in, plain, ct_out, flags=0):
    j = _job(plan, ct_in, plain, ct_out, flags)
    _chk(_lib.he_batch_rebind(b, index, ctypes.byref(j)), "he_batch_rebind")


def he_batch_run(b, stream=None):
    _chk(_lib.he_batch_run(b, _stream(stream)), "he_batch_run")


def he_batch_sync(b, stream=None):
    _chk(_lib.he_batch_sync(b, _stream(stream)), "he_batch_sync")


def he_batch_set_spin_limit(b, polls):
    _chk(_lib.he_batch_set_spin_limit(b, polls), "he_batch_set_spin_limit")


def he_batch_get_info(b):
    i = he_batch_info()
    _chk(_lib.he_batch_get_info(b, ctypes.byref(i)), "he_batch_get_info")
    return {n: getattr(i, n) for n, _ in he_batch_info._fields_}


def he_batch_destroy(b):
    _chk(_lib.he_batch_destroy(b), "he_batch_destroy")


# ------------------------------------------------------------------ serving
HE_SERVE_CONTINUOUS, HE_SERVE_SEQUENTIAL = 0, 1
HE_SERVE_KEEP_RESIDENT = 0x1


class he_server_params(ctypes.Structure):
    _fields_ = [("device", c_i32), ("mode", c_u32), ("mem_cap_bytes", c_u64), ("arena_bytes", c_u64),
                ("max_batch_jobs", c_u32), ("slots", c_u32), ("session_jobs", c_u32), ("poll_us", c_u32)]


class he_job_result(ctypes.Structure):
    _fields_ = [("status", c_i32), ("latency_s", ctypes.c_double), ("queue_s", ctypes.c_double)]


class he_server_info(ctypes.Structure):
    _fields_ = [("completed", c_u64), ("rejected", c_u64), ("epochs", c_u64), ("mean_jobs_per_epoch", ctypes.c_double),
                ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double), ("mean_s", ctypes.c_double),
                ("max_s", ctypes.c_double), ("span_s", ctypes.c_double), ("peak_bytes", c_u64),
                ("in_use_bytes", c_u64), ("single_epochs", c_u64), ("resident_hits", c_u64),
                ("resident_misses", c_u64), ("evictions", c_u64), ("fwd_planes", c_u64), ("failed", c_u64),
                ("resident_blocks", c_u64)]


def he_server_create(mem_cap_bytes=64 << 30, mode=HE_SERVE_CONTINUOUS, device=0, arena_bytes=0, max_batch_jobs=0,
                     slots=0, session_jobs=0, poll_us=0):
    p = he_server_params(device, mode, mem_cap_bytes, arena_bytes, max_batch_jobs, slots, session_jobs, poll_us)
    h = c_void_p()
    _chk(_lib.he_server_create(ctypes.byref(p), ctypes.byref(h)), "he_server_create")
    return h


def he_server_submit(s, ctx, plan, ct_in, plain, ct_out, flags=0, session=0, submit_flags=0):
    j = _job(plan, ct_in, plain, ct_out, flags)
    t = c_u64()
    _chk(_lib.he_server_submit(s, ctx, ctypes.byref(j), session, submit_flags, ctypes.byref(t)), "he_server_submit")
    return t.value


def he_server_wait(s, ticket, timeout_us=-1):
    r = he_job_result()
    st = _lib.he_server_wait(s, ticket, timeout_us, ctypes.byref(r))
    _chk(st, "he_server_wait")
    return dict(status=r.status, latency_s=r.latency_s, queue_s=r.queue_s)


def he_server_drain(s):
    _chk(_lib.he_server_drain(s), "he_server_drain")


def he_server_close_session(s, session):
    _chk(_lib.he_server_close_session(s, session), "he_server_close_session")


def he_server_replay(s, ctxs, jobs, arrival_s, sessions=None, submit_flags=0):
    """jobs: list of (plan, ct_in, plain, ct_out, flags); returns per-job latency (s)."""
    n = len(jobs)
    ctx_arr = (c_void_p * n)(*[c.value if isinstance(c, c_void_p) else c for c in ctxs])
    job_arr = (he_job * n)(*[_job(*j) for j in jobs])
    arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
    ses = None if sessions is None else np.ascontiguousarray(sessions, dtype=np.uint64)
    lat = np.zeros(n, dtype=np.float64)
    _chk(_lib.he_server_replay(s, n, ctypes.cast(ctx_arr, c_void_p), ctypes.cast(job_arr, c_void_p),
                               arr.ctypes.data_as(c_void_p), None if ses is None else ses.ctypes.data_as(c_void_p),
                               submit_flags, lat.ctypes.data_as(c_void_p)), "he_server_replay")
    return lat


def he_server_stats(s):
    i = he_server_info()
    _chk(_lib.he_server_stats(s, ctypes.byref(i)), "he_server_stats")
    return {n: getattr(i, n) for n, _ in he_server_info._fields_}


def he_server_destroy(s):
    _chk(_lib.he_server_destroy(s), "he_server_destroy")


# ------------------------------------------------------------------ helpers
def to_device_u64(a, device="cuda"):
    """numpy uint64 array -> contiguous torch.uint64 tensor on the GPU."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).to(device).view(torch.uint64)


def to_numpy_u64(t):
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


def empty_u64(shape, device="cuda"):
    return torch.empty(shape, dtype=torch.int64, device=device).view(torch.uint64)


def workspace(nbytes, device="cuda"):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class Context:
    """Owns an he_ctx handle."""

    def __init__(self, N, L, prime_bits=48, t=65537, q=None, arith=HE_ARITH_AUTO, device=0):
        self.h = he_ctx_create(N, L, prime_bits, t, q, arith, device)
        self.N, self.L, self.t, self.arith = he_ctx_info(self.h)
        self.q, self.psi = he_ctx_moduli(self.h, self.L)

    def close(self):
        if self.h:
            he_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Owns an he_plan handle: on a context, or (ctx None, N given) a host plan."""

    def __init__(self, ctx, kind, N=None, **shape):
        self.ctx = ctx
        self.shape = dict(shape)
        self.kind = kind
        self.h = he_plan_create(ctx.h, kind, **shape) if ctx is not None else he_plan_create_host(N, kind, **shape)
        self.info = he_plan_get_info(self.h)

    def workspace_size(self, flags=0):
        return he_workspace_size(self.h, flags)

    def close(self):
        if self.h:
            he_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
