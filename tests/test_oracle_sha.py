"""Pins of the oracle's SHA-2 / HMAC / MGF1 against independent sources.

- hashlib / hmac (an independent implementation) at every padding edge and
  at random lengths;
- the round constants and initial values re-derived from the primes
  (FIPS 180-4 Sections 4.2.2, 4.2.3, 5.3.3, 5.3.5);
- MGF1 prefix structure (RFC 8017 Appendix B.2.1).
"""
import hashlib
import hmac
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle

EDGE_LENGTHS = [0, 1, 3, 55, 56, 57, 63, 64, 65, 111, 112, 113, 119, 120, 127, 128, 129,
                191, 192, 255, 256, 1000]


@pytest.mark.parametrize("length", EDGE_LENGTHS)
def test_sha2_padding_edges(length):
    data = np.random.default_rng([101, length]).bytes(length)
    assert oracle.sha256(data) == hashlib.sha256(data).digest()
    assert oracle.sha512(data) == hashlib.sha512(data).digest()


def test_fips180_example_messages():
    # The example messages of FIPS 180 (one block, two blocks, a million 'a').
    # Expected digests come from hashlib at test time, not transcribed.
    msgs = [b"abc",
            b"abcdbcdecdefdefgefghfghighijhijkijkljklmklmnlmnomnopnopq",
            b"abcdefghbcdefghicdefghijdefghijkefghijklfghijklmghijklmnhijklmno"
            b"ijklmnopjklmnopqklmnopqrlmnopqrsmnopqrstnopqrstu",
            b"a" * 1000000]
    for m in msgs:
        assert oracle.sha256(m) == hashlib.sha256(m).digest()
        assert oracle.sha512(m) == hashlib.sha512(m).digest()


@settings(max_examples=60, deadline=None)
@given(st.binary(min_size=0, max_size=300))
def test_sha2_random(data):
    assert oracle.sha256(data) == hashlib.sha256(data).digest()
    assert oracle.sha512(data) == hashlib.sha512(data).digest()


@settings(max_examples=40, deadline=None)
@given(st.binary(min_size=0, max_size=200), st.binary(min_size=0, max_size=300))
def test_hmac_random(key, msg):
    assert oracle.hmac_sha256(key, msg) == hmac.new(key, msg, "sha256").digest()
    assert oracle.hmac_sha512(key, msg) == hmac.new(key, msg, "sha512").digest()


def _primes(count):
    out, c = [], 2
    while len(out) < count:
        if all(c % p for p in out if p * p <= c):
            out.append(c)
        c += 1
    return out


def _iroot(x, r):
    """floor(x ** (1/r)) for integers, by Newton iteration."""
    if x < 2:
        return x
    y = 1 << ((x.bit_length() + r - 1) // r)
    while True:
        z = ((r - 1) * y + x // y ** (r - 1)) // r
        if z >= y:
            return y
        y = z


def test_sha256_constants_from_primes():
    k, iv = oracle.sha256_constants()
    ps = _primes(64)
    # first 32 bits of the fractional parts of the cube roots of the first 64 primes
    assert k == [_iroot(p << 96, 3) & 0xFFFFFFFF for p in ps]
    # ... and of the square roots of the first 8 primes
    assert iv == [_iroot(p << 64, 2) & 0xFFFFFFFF for p in ps[:8]]


def test_sha512_constants_from_primes():
    k, iv = oracle.sha512_constants()
    ps = _primes(80)
    assert k == [_iroot(p << 192, 3) & 0xFFFFFFFFFFFFFFFF for p in ps]
    assert iv == [_iroot(p << 128, 2) & 0xFFFFFFFFFFFFFFFF for p in ps[:8]]


@pytest.mark.parametrize("seedlen", [0, 16, 48, 96])
def test_mgf1_structure(seedlen):
    seed = os.urandom(seedlen)
    long256 = oracle.mgf1_sha256(seed, 100)
    long512 = oracle.mgf1_sha512(seed, 200)
    # first output block is Hash(seed || 00000000) and the next Hash(seed || 00000001)
    assert long256[:32] == hashlib.sha256(seed + b"\0\0\0\0").digest()
    assert long256[32:64] == hashlib.sha256(seed + b"\0\0\0\1").digest()
    assert long512[:64] == hashlib.sha512(seed + b"\0\0\0\0").digest()
    assert long512[64:128] == hashlib.sha512(seed + b"\0\0\0\1").digest()
    # shorter outputs are prefixes of longer ones
    for L in (0, 1, 31, 33, 64, 99):
        assert oracle.mgf1_sha256(seed, L) == long256[:L]
    for L in (0, 1, 63, 65, 128, 199):
        assert oracle.mgf1_sha512(seed, L) == long512[:L]
