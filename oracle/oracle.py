"""ctypes wrapper of the C oracle (``liboracle.so``).

TEST INFRASTRUCTURE: see the package docstring.  Builds the library with gcc
on first use if it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "slh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

PARAM_IDS = {"128f": 1, "192f": 2, "256f": 3, "128s": 4, "192s": 5, "256s": 6,
             "shake-128f": 7, "shake-192f": 8, "shake-256f": 9, "shake-128s": 10, "shake-192s": 11,
             "shake-256s": 12}


def build(force: bool = True) -> str:
    """Compile slh_oracle.c into liboracle.so with gcc (plain -O2, no SIMD flags)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-Wall", "-Wextra",
             "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class or_params(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int) for f in
                ("n", "h", "d", "hp", "a", "k", "lg_w", "len1", "len2", "len", "m", "wide", "shake")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=False)
            L = ctypes.CDLL(_LIB)
            P = ctypes.POINTER(or_params)
            u8p = ctypes.c_char_p
            sz = ctypes.c_size_t
            L.or_params_get.argtypes = [ctypes.c_int, P]
            L.or_params_custom.argtypes = [ctypes.c_int] * 5 + [P]
            L.or_sig_bytes.argtypes = [P]
            L.or_sig_bytes.restype = sz
            L.or_shake256.argtypes = [u8p, sz, ctypes.c_void_p, sz]
            for fn in ("or_sha256", "or_sha512", "or_sha3_256"):
                getattr(L, fn).argtypes = [u8p, sz, ctypes.c_void_p]
            for fn in ("or_hmac_sha256", "or_hmac_sha512"):
                getattr(L, fn).argtypes = [u8p, sz, u8p, sz, ctypes.c_void_p]
            for fn in ("or_mgf1_sha256", "or_mgf1_sha512"):
                getattr(L, fn).argtypes = [u8p, sz, ctypes.c_void_p, sz]
            L.or_sha256_constants.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
            L.or_sha512_constants.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
            L.or_prf.argtypes = [P, u8p, u8p, u8p, ctypes.c_void_p]
            L.or_f.argtypes = [P, u8p, u8p, u8p, ctypes.c_void_p]
            L.or_h.argtypes = [P, u8p, u8p, u8p, ctypes.c_void_p]
            L.or_t.argtypes = [P, u8p, u8p, u8p, sz, ctypes.c_void_p]
            L.or_prf_msg.argtypes = [P, u8p, u8p, u8p, sz, ctypes.c_void_p]
            L.or_h_msg.argtypes = [P, u8p, u8p, u8p, u8p, sz, ctypes.c_void_p]
            L.or_base_2b.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
            L.or_wots_pkgen.argtypes = [P, u8p, u8p, u8p, ctypes.c_void_p]
            L.or_xmss_node.argtypes = [P, u8p, ctypes.c_uint32, ctypes.c_uint32, u8p, u8p,
                                       ctypes.c_void_p]
            L.or_fors_node.argtypes = [P, u8p, ctypes.c_uint32, ctypes.c_uint32, u8p, u8p,
                                       ctypes.c_void_p]
            L.or_fors_pk_from_sig.argtypes = [P, u8p, u8p, u8p, u8p, ctypes.c_void_p]
            L.or_xmss_pk_from_sig.argtypes = [P, ctypes.c_uint32, u8p, u8p, u8p, u8p,
                                              ctypes.c_void_p]
            L.or_split_digest.argtypes = [P, u8p, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_uint64),
                                          ctypes.POINTER(ctypes.c_uint32)]
            L.or_keygen.argtypes = [P, u8p, u8p, u8p, ctypes.c_void_p, ctypes.c_void_p]
            L.or_sign.argtypes = [P, u8p, sz, u8p, ctypes.c_char_p, ctypes.c_void_p]
            L.or_verify.argtypes = [P, u8p, sz, u8p, sz, u8p]
            L.or_encode_ext.argtypes = [u8p, sz, u8p, sz, ctypes.c_int, ctypes.c_void_p]
            L.or_encode_ext.restype = ctypes.c_long
            L.or_sign_ext.argtypes = [P, u8p, sz, u8p, sz, ctypes.c_int, u8p, ctypes.c_char_p, ctypes.c_void_p]
            L.or_verify_ext.argtypes = [P, u8p, sz, u8p, sz, ctypes.c_int, u8p, sz, u8p]
            L.or_counters_get.argtypes = [ctypes.c_void_p]
            _lib = L
    return _lib


def params(which) -> or_params:
    """Parameter struct for '128f' / '192f' / '256f' / '128s' / '192s' / '256s' (or ids 1..6)."""
    pid = PARAM_IDS.get(which, which)
    p = or_params()
    if lib().or_params_get(int(pid), ctypes.byref(p)) != 0:
        raise ValueError("unknown parameter set %r" % (which,))
    return p


def custom_params(n, h, d, a, k) -> or_params:
    p = or_params()
    if lib().or_params_custom(n, h, d, a, k, ctypes.byref(p)) != 0:
        raise ValueError("parameters outside the oracle's limits")
    return p


def _p(p):
    return ctypes.byref(p if isinstance(p, or_params) else params(p))


def sig_bytes(p) -> int:
    return lib().or_sig_bytes(_p(p))


def sha256(b: bytes) -> bytes:
    out = ctypes.create_string_buffer(32)
    lib().or_sha256(b, len(b), out)
    return out.raw


def shake256(b: bytes, outlen: int) -> bytes:
    out = ctypes.create_string_buffer(max(1, outlen))
    lib().or_shake256(b, len(b), out, outlen)
    return out.raw[:outlen]


def sha3_256(b: bytes) -> bytes:
    out = ctypes.create_string_buffer(32)
    lib().or_sha3_256(b, len(b), out)
    return out.raw


def sha512(b: bytes) -> bytes:
    out = ctypes.create_string_buffer(64)
    lib().or_sha512(b, len(b), out)
    return out.raw


def hmac_sha256(key: bytes, msg: bytes) -> bytes:
    out = ctypes.create_string_buffer(32)
    lib().or_hmac_sha256(key, len(key), msg, len(msg), out)
    return out.raw


def hmac_sha512(key: bytes, msg: bytes) -> bytes:
    out = ctypes.create_string_buffer(64)
    lib().or_hmac_sha512(key, len(key), msg, len(msg), out)
    return out.raw


def mgf1_sha256(seed: bytes, length: int) -> bytes:
    out = ctypes.create_string_buffer(max(length, 1))
    lib().or_mgf1_sha256(seed, len(seed), out, length)
    return out.raw[:length]


def mgf1_sha512(seed: bytes, length: int) -> bytes:
    out = ctypes.create_string_buffer(max(length, 1))
    lib().or_mgf1_sha512(seed, len(seed), out, length)
    return out.raw[:length]


def sha256_constants():
    k = (ctypes.c_uint32 * 64)()
    iv = (ctypes.c_uint32 * 8)()
    lib().or_sha256_constants(k, iv)
    return list(k), list(iv)


def sha512_constants():
    k = (ctypes.c_uint64 * 80)()
    iv = (ctypes.c_uint64 * 8)()
    lib().or_sha512_constants(k, iv)
    return list(k), list(iv)


def prf(p, pk_seed, sk_seed, adrs):
    p = p if isinstance(p, or_params) else params(p)
    out = ctypes.create_string_buffer(p.n)
    lib().or_prf(ctypes.byref(p), pk_seed, sk_seed, adrs, out)
    return out.raw


def F(p, pk_seed, adrs, m1):
    p = p if isinstance(p, or_params) else params(p)
    out = ctypes.create_string_buffer(p.n)
    lib().or_f(ctypes.byref(p), pk_seed, adrs, m1, out)
    return out.raw


def H(p, pk_seed, adrs, m2):
    p = p if isinstance(p, or_params) else params(p)
    out = ctypes.create_string_buffer(p.n)
    lib().or_h(ctypes.byref(p), pk_seed, adrs, m2, out)
    return out.raw


def T(p, pk_seed, adrs, ml):
    p = p if isinstance(p, or_params) else params(p)
    assert len(ml) % p.n == 0
    out = ctypes.create_string_buffer(p.n)
    lib().or_t(ctypes.byref(p), pk_seed, adrs, ml, len(ml) // p.n, out)
    return out.raw


def prf_msg(p, sk_prf, opt_rand, msg):
    p = p if isinstance(p, or_params) else params(p)
    out = ctypes.create_string_buffer(p.n)
    lib().or_prf_msg(ctypes.byref(p), sk_prf, opt_rand, msg, len(msg), out)
    return out.raw


def h_msg(p, r, pk_seed, pk_root, msg):
    p = p if isinstance(p, or_params) else params(p)
    out = ctypes.create_string_buffer(p.m)
    lib().or_h_msg(ctypes.byref(p), r, pk_seed, pk_root, msg, len(msg), out)
    return out.raw


def base_2b(x: bytes, b: int, out_len: int):
    out = (ctypes.c_uint32 * out_len)()
    lib().or_base_2b(x, b, out_len, out)
    return list(out)


def wots_pkgen(p, sk_seed, pk_seed, adrs):
    out = ctypes.create_string_buffer(p.n)
    lib().or_wots_pkgen(ctypes.byref(p), sk_seed, pk_seed, adrs, out)
    return out.raw


def xmss_node(p, sk_seed, i, z, pk_seed, adrs):
    out = ctypes.create_string_buffer(p.n)
    lib().or_xmss_node(ctypes.byref(p), sk_seed, i, z, pk_seed, adrs, out)
    return out.raw


def fors_node(p, sk_seed, i, z, pk_seed, adrs):
    out = ctypes.create_string_buffer(p.n)
    lib().or_fors_node(ctypes.byref(p), sk_seed, i, z, pk_seed, adrs, out)
    return out.raw


def fors_pk_from_sig(p, sig_fors, md, pk_seed, adrs):
    out = ctypes.create_string_buffer(p.n)
    lib().or_fors_pk_from_sig(ctypes.byref(p), sig_fors, md, pk_seed, adrs, out)
    return out.raw


def xmss_pk_from_sig(p, idx, sig_xmss, msg_n, pk_seed, adrs):
    out = ctypes.create_string_buffer(p.n)
    lib().or_xmss_pk_from_sig(ctypes.byref(p), idx, sig_xmss, msg_n, pk_seed, adrs, out)
    return out.raw


def split_digest(p, digest):
    md = ctypes.create_string_buffer(128)
    t = ctypes.c_uint64()
    l = ctypes.c_uint32()
    lib().or_split_digest(ctypes.byref(p), digest, md, ctypes.byref(t), ctypes.byref(l))
    return md.raw[:(p.k * p.a + 7) // 8], t.value, l.value


def keygen(p, seed: bytes):
    """seed = SK.seed | SK.prf | PK.seed (3n bytes) -> (pk 2n, sk 4n)."""
    p = p if isinstance(p, or_params) else params(p)
    n = p.n
    assert len(seed) == 3 * n
    sk = ctypes.create_string_buffer(4 * n)
    pk = ctypes.create_string_buffer(2 * n)
    rc = lib().or_keygen(ctypes.byref(p), seed[:n], seed[n:2 * n], seed[2 * n:], sk, pk)
    if rc != 0:
        raise ValueError("or_keygen failed")
    return pk.raw, sk.raw


def sign(p, msg: bytes, sk: bytes, addrnd: bytes | None = None) -> bytes:
    """Deterministic signature (opt_rand = PK.seed) unless addrnd is given."""
    p = p if isinstance(p, or_params) else params(p)
    out = ctypes.create_string_buffer(sig_bytes(p))
    rc = lib().or_sign(ctypes.byref(p), msg, len(msg), sk, addrnd, out)
    if rc != 0:
        raise ValueError("or_sign failed")
    return out.raw


def verify(p, msg: bytes, sig: bytes, pk: bytes) -> bool:
    p = p if isinstance(p, or_params) else params(p)
    rc = lib().or_verify(ctypes.byref(p), msg, len(msg), sig, len(sig), pk)
    if rc < 0:
        raise ValueError("or_verify failed")
    return rc == 1


# message encodings of the external interface (FIPS 205 Section 10)
PURE, PH_SHA256, PH_SHA512 = 0, 1, 2


def encode_ext(msg: bytes, ctx: bytes = b"", ph: int = PURE) -> bytes:
    """M' of slh_sign / hash_slh_sign (Algorithms 22 and 23)."""
    out = ctypes.create_string_buffer(2 + len(ctx) + max(len(msg), 75))
    n = lib().or_encode_ext(msg, len(msg), ctx, len(ctx), ph, out)
    if n < 0:
        raise ValueError("or_encode_ext: bad arguments")
    return out.raw[:n]


def sign_ext(p, msg: bytes, sk: bytes, ctx: bytes = b"", ph: int = PURE, addrnd: bytes | None = None) -> bytes:
    """slh_sign (ph = PURE) or hash_slh_sign (Algorithms 22 / 23)."""
    p = p if isinstance(p, or_params) else params(p)
    out = ctypes.create_string_buffer(sig_bytes(p))
    if lib().or_sign_ext(ctypes.byref(p), msg, len(msg), ctx, len(ctx), ph, sk, addrnd, out) != 0:
        raise ValueError("or_sign_ext failed")
    return out.raw


def verify_ext(p, msg: bytes, sig: bytes, pk: bytes, ctx: bytes = b"", ph: int = PURE) -> bool:
    p = p if isinstance(p, or_params) else params(p)
    rc = lib().or_verify_ext(ctypes.byref(p), msg, len(msg), ctx, len(ctx), ph, sig, len(sig), pk)
    if rc < 0:
        raise ValueError("or_verify_ext failed")
    return rc == 1


COUNTER_NAMES = ("F", "PRF", "H", "T", "sha256_blocks", "sha512_blocks", "PRF_msg", "H_msg", "keccak_f")


def counters_reset():
    lib().or_counters_reset()


def counters():
    out = (ctypes.c_uint64 * len(COUNTER_NAMES))()
    lib().or_counters_get(out)
    return dict(zip(COUNTER_NAMES, list(out)))


__all__ = [n for n in dir() if not n.startswith("_") and n not in (
    "annotations", "ctypes", "os", "subprocess", "threading")]
