"""Pins of the oracle's SHAKE instantiation (FIPS 205 Section 11.1): the
Keccak-f[1600] sponge against hashlib's SHA3-256 and SHAKE256 (an
independent implementation) at every rate boundary and for multi-block
squeezes; the SHAKE parameter sets (same shapes as the SHA2 ones); and full
signatures equal to the independent bottom-up implementation, which hashes
with hashlib.shake_256 and builds the full 32-byte addresses itself."""
import hashlib

import pytest

import oracle
import pyslh


@pytest.mark.parametrize("mlen", [0, 1, 8, 135, 136, 137, 271, 272, 273, 1000])
def test_keccak_sponge_matches_hashlib(mlen):
    m = bytes((i * 131 + 7) & 0xFF for i in range(mlen))
    assert oracle.sha3_256(m) == hashlib.sha3_256(m).digest()
    for outlen in (16, 32, 49, 136, 137, 300):
        assert oracle.shake256(m, outlen) == hashlib.shake_256(m).digest(outlen)


@pytest.mark.parametrize("i", range(6))
def test_shake_sets_share_shapes(i):
    sha2 = ["128f", "192f", "256f", "128s", "192s", "256s"][i]
    a, b = oracle.params(sha2), oracle.params("shake-" + sha2)
    da, db = a.as_dict(), b.as_dict()
    assert db.pop("shake") == 1 and da.pop("shake") == 0
    da.pop("wide"); db.pop("wide")
    assert da == db
    assert oracle.sig_bytes(a) == oracle.sig_bytes(b)


@pytest.mark.parametrize("P", [pyslh.P(n=16, h=4, d=2, a=3, k=4, shake=True),
                               pyslh.P(n=32, h=6, d=3, a=2, k=6, shake=True)])
def test_tiny_shake_signatures_equal(P):
    p = oracle.custom_params(P.n, P.h, P.d, P.a, P.k)
    p.shake = 1
    p.wide = 0
    seed = bytes((3 * i + 1) & 0xFF for i in range(3 * P.n))
    pk, sk = pyslh.keygen(P, seed)
    assert oracle.keygen(p, seed) == (pk, sk)
    for mlen in (0, 5, 200):
        msg = bytes(range(mlen))
        sig = oracle.sign(p, msg, sk)
        assert sig == pyslh.sign(P, msg, sk)
        assert oracle.verify(p, msg, sig, pk)


@pytest.mark.slow
@pytest.mark.parametrize("name", ["shake-128f", "shake-256f"])
def test_shake_full_size_equals_independent_implementation(name):
    P = pyslh.SETS[name]
    p = oracle.params(name)
    seed = bytes((11 * i + 5) & 0xFF for i in range(3 * p.n))
    pk, sk = oracle.keygen(p, seed)
    assert (pk, sk) == pyslh.keygen(P, seed)
    msg = b"shake parameter set"
    sig = oracle.sign(p, msg, sk)
    assert sig == pyslh.sign(P, msg, sk)
    assert oracle.verify(p, msg, sig, pk)
