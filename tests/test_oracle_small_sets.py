"""Pins of the oracle for the 'small' (-s) SHA2 parameter sets of FIPS 205:
the parameter table (Table 2 of the standard, tests/golden), the digest
length m and signature size from their formulas, internal consistency of a
full signature (every layer's root recomputed from the signature equals the
full-tree root, the last one PK.root), sign/verify round trips, and byte
equality with the independent bottom-up implementation (tests/pyslh.py)."""
import json
import os

import pytest

import oracle
import pyslh

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fips205_small_sets.json")))
SMALL = ["128s", "192s", "256s"]


@pytest.mark.parametrize("name", SMALL)
def test_small_param_table(name):
    p = oracle.params(name)
    g = GOLD[name]
    assert (p.n, p.h, p.d, p.hp, p.a, p.k, p.lg_w) == (g["n"], g["h"], g["d"], g["hp"], g["a"], g["k"], g["lg_w"])
    # m = ceil(k a / 8) + ceil((h - h') / 8) + ceil(h' / 8)  (FIPS 205 Algorithm 19)
    assert p.m == g["m"] == (p.k * p.a + 7) // 8 + (p.h - p.hp + 7) // 8 + (p.hp + 7) // 8
    assert oracle.sig_bytes(p) == g["sig_bytes"] == p.n * (1 + p.k * (p.a + 1) + p.h + p.d * p.len)
    assert 2 * p.n == g["pk_bytes"]


@pytest.mark.slow
@pytest.mark.parametrize("name", SMALL)
def test_small_full_size_equals_independent_implementation(name):
    P = pyslh.SETS[name]
    p = oracle.params(name)
    seed = bytes((7 * i + 3) & 0xFF for i in range(3 * p.n))
    pk, sk = oracle.keygen(p, seed)
    assert (pk, sk) == pyslh.keygen(P, seed)
    msg = b"small parameter set"
    sig = oracle.sign(p, msg, sk)
    assert sig == pyslh.sign(P, msg, sk)
    assert oracle.verify(p, msg, sig, pk)
    bad = bytearray(sig)
    bad[len(sig) // 2] ^= 1
    assert not oracle.verify(p, msg, bytes(bad), pk)
