"""Brute-force pins of the oracle on tiny parameter sets, and a byte-for-byte
comparison with the independently structured hashlib implementation at the
real parameter sets.

The tiny sets keep every tree small enough that all nodes are built
explicitly, level by level, from the F/H/PRF/T definitions; every auth path
for every leaf index and every FORS index is then checked against those
nodes, independently of the oracle's auth-path code.
"""
import itertools

import pytest

import oracle
import pyslh

TINY = [
    pyslh.P(n=16, h=4, d=2, a=3, k=4),   # SHA-256 everywhere
    pyslh.P(n=24, h=4, d=2, a=3, k=5),   # SHA-512 for H and T
    pyslh.P(n=32, h=6, d=3, a=2, k=6),
]


def _op(P):
    return oracle.custom_params(P.n, P.h, P.d, P.a, P.k)


def _adrs32(layer, tree, typ, w1=0, w2=0, w3=0):
    return (layer.to_bytes(4, "big") + tree.to_bytes(12, "big") + typ.to_bytes(4, "big")
            + w1.to_bytes(4, "big") + w2.to_bytes(4, "big") + w3.to_bytes(4, "big"))


@pytest.mark.parametrize("P", TINY, ids=lambda P: "n%d_h%d_d%d_a%d_k%d" % (P.n, P.h, P.d, P.a, P.k))
def test_tiny_every_node(P):
    p = _op(P)
    assert (p.len, p.m) == (P.len, P.m)
    seed = bytes((3 * i + 1) & 0xFF for i in range(3 * P.n))
    sk_seed, pk_seed = seed[:P.n], seed[2 * P.n:]
    hs = pyslh.Hashes(P, pk_seed)
    # keygen: top tree root
    pk_o, sk_o = oracle.keygen(p, seed)
    assert (pk_o, sk_o) == pyslh.keygen(P, seed)
    # every XMSS node of two trees on every layer against the oracle's node function
    for layer in range(P.d):
        for tree in (0, 1, (1 << (P.h - (layer + 1) * P.hp)) - 1 if layer < P.d - 1 else 0):
            xt = pyslh.XmssTree(hs, sk_seed, layer, tree)
            a = _adrs32(layer, tree, 0)
            for z, level in enumerate(xt.levels):
                for i, node in enumerate(level):
                    assert oracle.xmss_node(p, sk_seed, i, z, pk_seed, a) == node
            # WOTS+ signature of every leaf for a few messages: pkFromSig gives the leaf,
            # and the climb through the auth path gives the root
            for leaf in range(1 << P.hp):
                for msg_n in (bytes(P.n), bytes([0xFF]) * P.n, bytes(range(P.n))):
                    sx = xt.sign(msg_n, leaf)
                    assert oracle.xmss_pk_from_sig(p, leaf, sx, msg_n, pk_seed, a) == xt.root
    # every FORS node for two keypair addresses
    for tree, kp in ((0, 0), (5, (1 << P.hp) - 1)):
        ff = pyslh.ForsForest(hs, sk_seed, tree, kp)
        a = _adrs32(0, tree, 3, kp)
        for z, level in enumerate(ff.levels):
            for i, node in enumerate(level):
                assert oracle.fors_node(p, sk_seed, i, z, pk_seed, a) == node
        # every index of every tree: pkFromSig of the brute-force signature gives the pk
        t = 1 << P.a
        for idx in range(t):
            md_bits = "".join(format(idx, "0%db" % P.a) for _ in range(P.k))
            md_bits += "0" * ((-len(md_bits)) % 8)
            md = int(md_bits, 2).to_bytes(len(md_bits) // 8, "big")
            assert pyslh.indices_of(md, P.a, P.k) == [idx] * P.k
            assert oracle.fors_pk_from_sig(p, ff.sign(md), md, pk_seed, a) == ff.pk


@pytest.mark.parametrize("P", TINY, ids=lambda P: "n%d" % P.n)
def test_tiny_signatures_equal(P):
    p = _op(P)
    seed = bytes((5 * i + 2) & 0xFF for i in range(3 * P.n))
    pk, sk = pyslh.keygen(P, seed)
    for mlen in (0, 1, 31, 64, 200):
        msg = bytes((i * 11) & 0xFF for i in range(mlen))
        sig = oracle.sign(p, msg, sk)
        assert sig == pyslh.sign(P, msg, sk)
        assert oracle.verify(p, msg, sig, pk)


def test_tiny_all_leaf_indices_reached():
    """Over many messages, every idx_leaf and several idx_tree values occur,
    and the oracle agrees with the brute-force signature for each."""
    P = TINY[0]
    p = _op(P)
    seed = bytes(range(3 * P.n))
    pk, sk = pyslh.keygen(P, seed)
    seen = set()
    for i in itertools.count():
        msg = i.to_bytes(4, "big")
        keep = {}
        ref = pyslh.sign(P, msg, sk, keep=keep)
        assert oracle.sign(p, msg, sk) == ref
        seen.add((keep["idx_tree"], keep["idx_leaf"]))
        if len({l for _, l in seen}) == 1 << P.hp and len({t for t, _ in seen}) >= 2 or i > 200:
            break
    assert len({l for _, l in seen}) == 1 << P.hp


@pytest.mark.parametrize("name", ["128f", "192f", "256f"])
def test_full_size_equals_independent_implementation(name):
    P = pyslh.SETS[name]
    p = oracle.params(name)
    from paper_2512_23969_amd import workloads
    seed = workloads.key_seed(workloads.ID_OF[name], 1)
    pk, sk = oracle.keygen(p, seed)
    assert (pk, sk) == pyslh.keygen(P, seed)
    msg = workloads.messages(9, 1, 57)[0]
    assert oracle.sign(p, msg, sk) == pyslh.sign(P, msg, sk)
