"""CPU checks of the C-ABI library: it loads, exports every function that
include/slh.h declares, reports sizes, and rejects bad arguments before
touching a GPU.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2512_23969_amd import slh
    return slh


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "slh.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(slh_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("slh_keygen", "slh_sign_batch", "slh_verify", "slh_params", "slh_ctx_create",
              "slh_ctx_destroy", "slh_ctx_add_keys", "slh_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol():
    slh = _lib()
    for name in declared_functions():
        assert hasattr(slh.lib, name), name


def test_no_oracle_symbols_in_product_library():
    slh = _lib()
    for name in ("or_sign", "or_sha256", "or_keygen"):
        with pytest.raises(AttributeError):
            getattr(slh.lib, name)


SIZES = [(1, 16, 17088), (2, 24, 35664), (3, 32, 49856), (4, 16, 7856), (5, 24, 16224), (6, 32, 29792)]


@pytest.mark.parametrize("param,n,sig", SIZES + [(p + 6, n, sig) for p, n, sig in SIZES])
def test_sizes(param, n, sig):
    import oracle
    slh = _lib()
    s = slh.sizes(param)
    p = oracle.params(slh.NAMES[param])
    assert s["n"] == n and s["sig_bytes"] == sig == oracle.sig_bytes(p)
    assert (s["h"], s["d"], s["hp"], s["a"], s["k"], s["len"], s["m"]) == (p.h, p.d, p.hp, p.a, p.k, p.len, p.m)
    assert (s["seed_bytes"], s["pk_bytes"], s["sk_bytes"]) == (3 * n, 2 * n, 4 * n)


def test_bad_arguments_rejected_on_host():
    slh = _lib()
    L = slh.lib
    assert L.slh_params(13, ctypes.byref(slh.slh_sizes())) == slh.EINVAL
    assert L.slh_params(0, ctypes.byref(slh.slh_sizes())) == slh.EINVAL
    assert L.slh_params(1, None) == slh.EINVAL
    assert L.slh_keygen(9, b"x" * 48, None, None) == slh.EINVAL
    assert L.slh_keygen(1, None, None, None) == slh.EINVAL
    assert L.slh_verify(0, b"", 0, b"", 0, b"") == slh.EINVAL
    # a wrong signature length is "invalid", decided before any device work
    assert L.slh_verify(1, b"m", 1, b"s" * 10, 10, b"p" * 32) == 0
    assert L.slh_ctx_create(0, 0, None) == slh.EINVAL
    assert L.slh_sign_batch(None, None, 0, None, 0, None, 0, 0, None) == slh.EINVAL
    assert L.slh_ctx_destroy(None) == 0
    assert isinstance(L.slh_last_error(None), bytes)
