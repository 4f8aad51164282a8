"""Structural pins of the oracle: the paper's printed sizes and counts, the
closed forms of base_2b and the digest split, internal consistency
(public keys and roots recomputed from signatures), sign -> verify round
trips and rejection of every single-field corruption.
"""
import json
import os

import pytest

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_figures.json")))
SETS = ["128f", "192f", "256f"]


@pytest.mark.parametrize("name", SETS)
def test_param_table_matches_paper(name):
    p = oracle.params(name)
    g = GOLD["param_sets"][name]
    assert (p.n, p.h, p.d, p.a, p.k, 1 << p.lg_w) == (g["n"], g["h"], g["d"], g["log_t"], g["k"], g["w"])
    assert p.hp * p.d == p.h


def test_signature_size_128f_matches_paper():
    assert oracle.sig_bytes(oracle.params("128f")) == GOLD["sig_bytes_128f"]["value"]


@pytest.mark.parametrize("name", SETS)
def test_tree_counts_match_paper(name):
    p = oracle.params(name)
    assert p.d * (1 << p.hp) == GOLD["hypertree_leaves"][name]
    assert p.k * (1 << p.a) == GOLD["fors_leaves"][name]
    assert p.k * (1 << p.a) * p.n == GOLD["fors_node_kib"][name] * 1024
    if name in GOLD["hypertree_node_kib"]:
        assert p.d * (1 << p.hp) * p.n == GOLD["hypertree_node_kib"][name] * 1024


@pytest.mark.parametrize("name", SETS)
def test_hashes_per_wots_leaf_match_paper(name):
    # one WOTS+ key generation = len PRF calls + len*(w-1) F calls
    p = oracle.params(name)
    oracle.counters_reset()
    oracle.wots_pkgen(p, bytes(p.n), bytes(range(p.n)), bytes(32))
    c = oracle.counters()
    assert c["PRF"] + c["F"] == GOLD["hashes_per_wots_leaf"][name]
    assert c["T"] == 1


def test_more_than_100k_hashes_per_128f_signature():
    p = oracle.params("128f")
    pk, sk = oracle.keygen(p, bytes(range(48)))
    oracle.counters_reset()
    oracle.sign(p, b"m", sk)
    c = oracle.counters()
    assert c["F"] + c["PRF"] + c["H"] + c["T"] > GOLD["min_hash_calls_per_signature"]["value"]


def test_derived_lengths():
    # m = ceil(k a / 8) + ceil((h - h/d) / 8) + ceil(h / 8d), len2 = 3 for w = 16
    want = {"128f": (34, 32, 3), "192f": (42, 48, 3), "256f": (49, 64, 3)}
    for name, (m, len1, len2) in want.items():
        p = oracle.params(name)
        assert (p.m, p.len1, p.len2, p.len) == (m, len1, len2, len1 + len2)


def test_base_2b_special_cases():
    x = bytes([0xA5, 0x3C, 0xF0, 0x0F])
    assert oracle.base_2b(x, 8, 4) == list(x)
    assert oracle.base_2b(x, 4, 8) == [0xA, 0x5, 0x3, 0xC, 0xF, 0x0, 0x0, 0xF]
    bits = [int(b) for byte in x for b in format(byte, "08b")]
    assert oracle.base_2b(x, 1, 32) == bits
    # 12-bit groups of a 3-byte string, most-significant first
    assert oracle.base_2b(bytes([0x12, 0x34, 0x56]), 12, 2) == [0x123, 0x456]
    # 6-bit groups: 0b000100 100011 010001 010110
    assert oracle.base_2b(bytes([0x12, 0x34, 0x56]), 6, 4) == [4, 35, 17, 22]
    # 9-bit groups over 4 bytes: the top 27 bits in three pieces
    v = int.from_bytes(x, "big")
    assert oracle.base_2b(x, 9, 3) == [(v >> (32 - 9 * (i + 1))) & 511 for i in range(3)]


@pytest.mark.parametrize("name", SETS)
def test_split_digest(name):
    p = oracle.params(name)
    digest = bytes((7 * i + 3) & 0xFF for i in range(p.m))
    md, t, l = oracle.split_digest(p, digest)
    mdb = (p.k * p.a + 7) // 8
    tb = (p.h - p.hp + 7) // 8
    assert md == digest[:mdb]
    assert t == int.from_bytes(digest[mdb:mdb + tb], "big") % (1 << (p.h - p.hp))
    assert l == digest[mdb + tb] % (1 << p.hp)
    if name == "256f":
        assert p.h - p.hp == 64  # all 64 bits of the tree index are used


def _keys(name, i=0):
    from paper_2512_23969_amd import workloads
    p = oracle.params(name)
    seed = workloads.key_seed(workloads.ID_OF[name], i)
    pk, sk = oracle.keygen(p, seed)
    return p, pk, sk


@pytest.mark.parametrize("name", SETS)
def test_sign_verify_roundtrip_and_corruptions(name):
    p, pk, sk = _keys(name)
    n = p.n
    msg = b"the quick brown fox"
    sig = oracle.sign(p, msg, sk)
    assert len(sig) == oracle.sig_bytes(p)
    assert oracle.verify(p, msg, sig, pk)
    assert oracle.sign(p, msg, sk) == sig  # deterministic
    # a different opt_rand gives a different R and still verifies
    sig2 = oracle.sign(p, msg, sk, addrnd=bytes(n))
    assert sig2[:n] != sig[:n] and oracle.verify(p, msg, sig2, pk)
    # every section of the signature is checked
    fors = n
    ht = n + p.k * (p.a + 1) * n
    xmss = (p.len + p.hp) * n
    offsets = {
        "R": 0, "fors_sk0": fors, "fors_auth0": fors + n,
        "fors_last_auth": ht - 1,
        "wots_layer0": ht, "auth_layer0": ht + p.len * n,
        "wots_top": ht + (p.d - 1) * xmss + 5 * n, "auth_top": ht + p.d * xmss - 1,
    }
    for where, off in offsets.items():
        bad = bytearray(sig)
        bad[off] ^= 0x01
        assert not oracle.verify(p, msg, bytes(bad), pk), where
    assert not oracle.verify(p, msg + b"!", sig, pk)
    assert not oracle.verify(p, msg, sig[:-1], pk)
    bad_pk = bytearray(pk)
    bad_pk[0] ^= 0x80
    assert not oracle.verify(p, msg, sig, bytes(bad_pk))
    bad_pk = bytearray(pk)
    bad_pk[-1] ^= 0x80
    assert not oracle.verify(p, msg, sig, bytes(bad_pk))


def _adrs(layer=0, tree=0, typ=0, w1=0, w2=0, w3=0):
    return (layer.to_bytes(4, "big") + tree.to_bytes(12, "big") + typ.to_bytes(4, "big")
            + w1.to_bytes(4, "big") + w2.to_bytes(4, "big") + w3.to_bytes(4, "big"))


@pytest.mark.parametrize("name", ["128f", "256f"])
def test_internal_consistency(name):
    """FORS pk and every layer root recomputed from the signature equal the
    values built from the complete trees with the node functions."""
    p, pk, sk = _keys(name)
    n = p.n
    sk_seed, pk_seed, pk_root = sk[:n], sk[2 * n:3 * n], sk[3 * n:]
    msg = bytes(range(40))
    sig = oracle.sign(p, msg, sk)
    r = sig[:n]
    md, idx_tree, idx_leaf = oracle.split_digest(p, oracle.h_msg(p, r, pk_seed, pk_root, msg))
    fors_adrs = _adrs(0, idx_tree, 3, idx_leaf)
    sig_fors = sig[n:n + p.k * (p.a + 1) * n]
    pk_fors = oracle.fors_pk_from_sig(p, sig_fors, md, pk_seed, fors_adrs)
    roots = b"".join(oracle.fors_node(p, sk_seed, t, p.a, pk_seed, fors_adrs) for t in range(p.k))
    assert pk_fors == oracle.T(p, pk_seed, _adrs(0, idx_tree, 4, idx_leaf), roots)
    # hypertree: layer j signs the previous root; check each root both ways
    m_j, tree, leaf = pk_fors, idx_tree, idx_leaf
    base = n + len(sig_fors)
    xb = (p.len + p.hp) * n
    for j in range(p.d):
        a = _adrs(j, tree)
        sx = sig[base + j * xb: base + (j + 1) * xb]
        r_sig = oracle.xmss_pk_from_sig(p, leaf, sx, m_j, pk_seed, a)
        if j in (0, 1, p.d - 1):  # full-tree recomputation is slow; check three layers
            assert r_sig == oracle.xmss_node(p, sk_seed, 0, p.hp, pk_seed, a)
        m_j = r_sig
        leaf, tree = tree & ((1 << p.hp) - 1), tree >> p.hp
    assert m_j == pk_root
