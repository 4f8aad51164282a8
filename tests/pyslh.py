"""Second, independently structured SPHINCS+ implementation on hashlib.

TEST INFRASTRUCTURE.  Used only to cross-check the C oracle.  It is written
bottom-up (every node of every tree is materialised in a list, level by
level) rather than with the recursive node functions of the C oracle, and
it hashes with Python's hashlib/hmac instead of the oracle's own SHA-2, so
a transcription slip in either one shows up as a byte difference.

Definitions followed: FIPS 205 Sections 4-9, 11.1 (SHAKE) and 11.2 (SHA2), the
paper's Section II-A description of WOTS+, FORS, XMSS and the hypertree, and
the Fig. 2 signing listing (leaf index = tree mod 2^h', tree >>= h').
"""
from __future__ import annotations

import hashlib
import hmac
from dataclasses import dataclass


@dataclass(frozen=True)
class P:
    n: int
    h: int
    d: int
    a: int
    k: int
    lg_w: int = 4
    shake: bool = False  # FIPS 205 Section 11.1: every hash is SHAKE256

    @property
    def hp(self):
        return self.h // self.d

    @property
    def w(self):
        return 1 << self.lg_w

    @property
    def len1(self):
        return (8 * self.n + self.lg_w - 1) // self.lg_w

    @property
    def len2(self):
        # smallest number of base-w digits whose range exceeds len1*(w-1)
        top = self.len1 * (self.w - 1)
        digits = 1
        while self.w ** digits <= top:
            digits += 1
        return digits

    @property
    def len(self):
        return self.len1 + self.len2

    @property
    def m(self):
        return (-(-self.k * self.a // 8)) + (-(-(self.h - self.hp) // 8)) + (-(-self.hp // 8))

    @property
    def wide(self):
        return self.n >= 24

    @property
    def sig_bytes(self):
        return self.n * (1 + self.k * (self.a + 1) + self.h + self.d * self.len)


SETS = {
    "128f": P(16, 66, 22, 6, 33),
    "192f": P(24, 66, 22, 8, 33),
    "256f": P(32, 68, 17, 9, 35),
    "128s": P(16, 63, 7, 12, 14),
    "192s": P(24, 63, 7, 14, 17),
    "256s": P(32, 64, 8, 14, 22),
    "shake-128f": P(16, 66, 22, 6, 33, shake=True),
    "shake-192f": P(24, 66, 22, 8, 33, shake=True),
    "shake-256f": P(32, 68, 17, 9, 35, shake=True),
    "shake-128s": P(16, 63, 7, 12, 14, shake=True),
    "shake-192s": P(24, 63, 7, 14, 17, shake=True),
    "shake-256s": P(32, 64, 8, 14, 22, shake=True),
}

# address types
WOTS_HASH, WOTS_PK, TREE, FORS_TREE, FORS_ROOTS, WOTS_PRF, FORS_PRF = range(7)


def adrs_c(layer: int, tree: int, typ: int, w1: int = 0, w2: int = 0, w3: int = 0) -> bytes:
    """22-byte compressed address: 1 byte layer, 8 bytes tree, 1 byte type, 3 words."""
    return (bytes([layer & 0xFF]) + tree.to_bytes(8, "big") + bytes([typ & 0xFF])
            + w1.to_bytes(4, "big") + w2.to_bytes(4, "big") + w3.to_bytes(4, "big"))


class Hashes:
    def __init__(self, p: P, pk_seed: bytes):
        self.p = p
        self.pk_seed = pk_seed
        self.calls = 0

    def _th(self, wide: bool, ac: bytes, data: bytes) -> bytes:
        self.calls += 1
        n = self.p.n
        if self.p.shake:
            # the full 32-byte address: 4-byte layer, 12-byte tree, 4-byte type, 3 words
            full = bytes(3) + ac[0:1] + bytes(4) + ac[1:9] + bytes(3) + ac[9:10] + ac[10:22]
            return hashlib.shake_256(self.pk_seed + full + data).digest(n)
        if wide:
            return hashlib.sha512(self.pk_seed + bytes(128 - n) + ac + data).digest()[:n]
        return hashlib.sha256(self.pk_seed + bytes(64 - n) + ac + data).digest()[:n]

    def F(self, ac, x):
        return self._th(False, ac, x)

    def PRF(self, ac, sk_seed):
        return self._th(False, ac, sk_seed)

    def H(self, ac, lr):
        return self._th(self.p.wide, ac, lr)

    def T(self, ac, blob):
        return self._th(self.p.wide, ac, blob)


def digits_of(p: P, msg_n: bytes):
    """base-16 digits of an n-byte value followed by the 3 checksum digits."""
    d = []
    for byte in msg_n:
        d.append(byte >> 4)
        d.append(byte & 15)
    d = d[:p.len1]
    csum = sum(p.w - 1 - x for x in d)
    shift = (8 - (p.len2 * p.lg_w) % 8) % 8
    csum <<= shift
    nbytes = (p.len2 * p.lg_w + 7) // 8
    cb = csum.to_bytes(nbytes, "big")
    cd = []
    for byte in cb:
        cd.append(byte >> 4)
        cd.append(byte & 15)
    return d + cd[:p.len2]


def indices_of(md: bytes, a: int, k: int):
    """k integers of a bits each, read most-significant bit first."""
    v = int.from_bytes(md, "big")
    total_bits = 8 * len(md)
    out = []
    for i in range(k):
        shift = total_bits - (i + 1) * a
        out.append((v >> shift) & ((1 << a) - 1))
    return out


class XmssTree:
    """All chains, leaves and nodes of one XMSS tree, built bottom-up."""

    def __init__(self, hs: Hashes, sk_seed: bytes, layer: int, tree: int):
        p = hs.p
        self.p, self.hs, self.layer, self.tree = p, hs, layer, tree
        self.chains = []      # chains[leaf][i] = list of w values (steps 0..w-1)
        leaves = []
        for leaf in range(1 << p.hp):
            per_leaf = []
            ends = b""
            for i in range(p.len):
                v = hs.PRF(adrs_c(layer, tree, WOTS_PRF, leaf, i, 0), sk_seed)
                vals = [v]
                for j in range(p.w - 1):
                    v = hs.F(adrs_c(layer, tree, WOTS_HASH, leaf, i, j), v)
                    vals.append(v)
                per_leaf.append(vals)
                ends += v
            self.chains.append(per_leaf)
            leaves.append(hs.T(adrs_c(layer, tree, WOTS_PK, leaf), ends))
        self.levels = [leaves]
        for z in range(1, p.hp + 1):
            below = self.levels[-1]
            self.levels.append([hs.H(adrs_c(layer, tree, TREE, 0, z, i), below[2 * i] + below[2 * i + 1])
                                for i in range(len(below) // 2)])

    @property
    def root(self):
        return self.levels[-1][0]

    def sign(self, msg_n: bytes, leaf: int) -> bytes:
        dg = digits_of(self.p, msg_n)
        wots = b"".join(self.chains[leaf][i][dg[i]] for i in range(self.p.len))
        auth = b"".join(self.levels[j][(leaf >> j) ^ 1] for j in range(self.p.hp))
        return wots + auth


class ForsForest:
    """All leaves and nodes of the k FORS trees of one keypair address."""

    def __init__(self, hs: Hashes, sk_seed: bytes, tree: int, keypair: int):
        p = hs.p
        self.p = p
        t = 1 << p.a
        self.sk = [hs.PRF(adrs_c(0, tree, FORS_PRF, keypair, 0, g), sk_seed) for g in range(p.k * t)]
        level0 = [hs.F(adrs_c(0, tree, FORS_TREE, keypair, 0, g), self.sk[g]) for g in range(p.k * t)]
        self.levels = [level0]
        for z in range(1, p.a + 1):
            below = self.levels[-1]
            self.levels.append([hs.H(adrs_c(0, tree, FORS_TREE, keypair, z, i), below[2 * i] + below[2 * i + 1])
                                for i in range(len(below) // 2)])
        roots = b"".join(self.levels[p.a])
        self.pk = hs.T(adrs_c(0, tree, FORS_ROOTS, keypair), roots)

    def sign(self, md: bytes) -> bytes:
        p = self.p
        out = b""
        for i, idx in enumerate(indices_of(md, p.a, p.k)):
            out += self.sk[(i << p.a) + idx]
            for j in range(p.a):
                out += self.levels[j][(i << (p.a - j)) + ((idx >> j) ^ 1)]
        return out


def prf_msg(p: P, sk_prf, opt_rand, msg):
    if p.shake:
        return hashlib.shake_256(sk_prf + opt_rand + msg).digest(p.n)
    alg = "sha512" if p.wide else "sha256"
    return hmac.new(sk_prf, opt_rand + msg, alg).digest()[:p.n]


def h_msg(p: P, r, pk_seed, pk_root, msg):
    if p.shake:
        return hashlib.shake_256(r + pk_seed + pk_root + msg).digest(p.m)
    H = hashlib.sha512 if p.wide else hashlib.sha256
    seed = r + pk_seed + H(r + pk_seed + pk_root + msg).digest()
    out = b""
    ctr = 0
    while len(out) < p.m:
        out += H(seed + ctr.to_bytes(4, "big")).digest()
        ctr += 1
    return out[:p.m]


def split(p: P, digest: bytes):
    mdb = -(-p.k * p.a // 8)
    tb = -(-(p.h - p.hp) // 8)
    lb = -(-p.hp // 8)
    md = digest[:mdb]
    idx_tree = int.from_bytes(digest[mdb:mdb + tb], "big") % (1 << (p.h - p.hp))
    idx_leaf = int.from_bytes(digest[mdb + tb:mdb + tb + lb], "big") % (1 << p.hp)
    return md, idx_tree, idx_leaf


def keygen(p: P, seed: bytes):
    n = p.n
    sk_seed, sk_prf, pk_seed = seed[:n], seed[n:2 * n], seed[2 * n:3 * n]
    hs = Hashes(p, pk_seed)
    root = XmssTree(hs, sk_seed, p.d - 1, 0).root
    return pk_seed + root, sk_seed + sk_prf + pk_seed + root


def sign(p: P, msg: bytes, sk: bytes, addrnd: bytes | None = None, keep=None) -> bytes:
    """Signature built from fully materialised trees.  If keep is a dict, the
    FORS forest and the XMSS trees are stored in it for inspection."""
    n = p.n
    sk_seed, sk_prf, pk_seed, pk_root = sk[:n], sk[n:2 * n], sk[2 * n:3 * n], sk[3 * n:4 * n]
    hs = Hashes(p, pk_seed)
    r = prf_msg(p, sk_prf, addrnd if addrnd is not None else pk_seed, msg)
    md, idx_tree, idx_leaf = split(p, h_msg(p, r, pk_seed, pk_root, msg))
    forest = ForsForest(hs, sk_seed, idx_tree, idx_leaf)
    out = r + forest.sign(md)
    m_j = forest.pk
    tree, leaf = idx_tree, idx_leaf
    trees = []
    for layer in range(p.d):
        xt = XmssTree(hs, sk_seed, layer, tree)
        trees.append(xt)
        out += xt.sign(m_j, leaf)
        m_j = xt.root
        leaf = tree & ((1 << p.hp) - 1)
        tree >>= p.hp
    if keep is not None:
        keep.update(forest=forest, trees=trees, md=md, idx_tree=idx_tree, idx_leaf=idx_leaf,
                    hash_calls=hs.calls)
    return out
