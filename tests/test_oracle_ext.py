"""Pins of the oracle's external interface (FIPS 205 Section 10): pure
SLH-DSA with a context string (Algorithms 22 / 24), HashSLH-DSA with SHA-256
or SHA-512 pre-hashing (Algorithms 23 / 25) and hedged signing (fresh
opt_rand, Algorithm 19 with addrnd).

What pins it: the hash-function identifiers are re-derived here from their
dotted OIDs with a DER encoder written from the X.690 rules; the pre-hash is
checked against hashlib; domain separation (a signature is valid for exactly
its own context string and encoding) and the deterministic special case
(addrnd = PK.seed) are properties the definitions imply."""
import hashlib

import pytest

import oracle

TINY = dict(n=16, h=4, d=2, a=3, k=5)


def der_oid(dotted: str) -> bytes:
    """X.690 encoding of an OBJECT IDENTIFIER: tag 0x06, length, then the
    first two arcs as 40 * a + b and every arc in base 128, high bit set on
    all but the last octet of an arc."""
    arcs = [int(x) for x in dotted.split(".")]
    vals = [40 * arcs[0] + arcs[1]] + arcs[2:]
    body = b""
    for v in vals:
        octs = [v & 0x7F]
        v >>= 7
        while v:
            octs.append(0x80 | (v & 0x7F))
            v >>= 7
        body += bytes(reversed(octs))
    return bytes([0x06, len(body)]) + body


@pytest.fixture(scope="module")
def tiny():
    p = oracle.custom_params(**TINY)
    pk, sk = oracle.keygen(p, bytes(range(3 * p.n)))
    return p, pk, sk


def test_prehash_encoding_oid_and_digest():
    m, ctx = b"message to pre-hash" * 7, b"app-context"
    for ph, oid, h in ((oracle.PH_SHA256, "2.16.840.1.101.3.4.2.1", hashlib.sha256),
                       (oracle.PH_SHA512, "2.16.840.1.101.3.4.2.3", hashlib.sha512)):
        enc = oracle.encode_ext(m, ctx, ph)
        assert enc[0] == 1 and enc[1] == len(ctx) and enc[2:2 + len(ctx)] == ctx
        o = der_oid(oid)
        assert len(o) == 11
        assert enc[2 + len(ctx):2 + len(ctx) + 11] == o
        assert enc[2 + len(ctx) + 11:] == h(m).digest()


def test_pure_encoding_lengths_and_limits():
    for mlen in (0, 1, 75, 300):
        for clen in (0, 1, 255):
            enc = oracle.encode_ext(bytes(mlen), bytes(clen), oracle.PURE)
            assert len(enc) == 2 + clen + mlen and enc[0] == 0 and enc[1] == clen
    with pytest.raises(ValueError):
        oracle.encode_ext(b"x", bytes(256), oracle.PURE)
    with pytest.raises(ValueError):
        oracle.encode_ext(b"x", b"", 3)


def test_domain_separation(tiny):
    p, pk, sk = tiny
    m = b"the same message"
    sigs = {}
    for ph in (oracle.PURE, oracle.PH_SHA256, oracle.PH_SHA512):
        for ctx in (b"", b"A", b"B"):
            sig = oracle.sign_ext(p, m, sk, ctx, ph)
            sigs[(ph, ctx)] = sig
            for ph2 in (oracle.PURE, oracle.PH_SHA256, oracle.PH_SHA512):
                for ctx2 in (b"", b"A", b"B"):
                    assert oracle.verify_ext(p, m, sig, pk, ctx2, ph2) == (ph2 == ph and ctx2 == ctx)
            # an external signature is not an internal one of the raw message
            assert not oracle.verify(p, m, sig, pk)
    assert len(set(sigs.values())) == len(sigs)


def test_hedged_signing(tiny):
    p, pk, sk = tiny
    n = p.n
    m = b"hedged"
    det = oracle.sign_ext(p, m, sk, b"c")
    # opt_rand = PK.seed is the deterministic variant
    assert oracle.sign_ext(p, m, sk, b"c", addrnd=pk[:n]) == det
    r1 = oracle.sign_ext(p, m, sk, b"c", addrnd=bytes([7]) * n)
    r2 = oracle.sign_ext(p, m, sk, b"c", addrnd=bytes([8]) * n)
    assert r1[:n] != det[:n] and r1[:n] != r2[:n]  # R depends on opt_rand
    for s in (r1, r2):
        assert oracle.verify_ext(p, m, s, pk, b"c")
