"""Work accounting of the signing path: hash compressions per signature and
per kernel, and the algorithmic 32-bit VALU operations they stand for.

Counts follow from the parameter sets (the paper's Table 1) and the SHA2
instantiation of the tweakable hashes: after the per-key PK.seed block,
F and PRF take one SHA-256 compression; H takes one SHA-256 (n = 16) or
SHA-512 (n >= 24) compression; T_l takes ceil((22 + l n + pad) / block)
compressions.  The paper gives the per-leaf figures 560 / 816 / 1072
(Section III-C) and the leaf counts (Section III-B) these reproduce.

VALU operations per compression.  The roofline uses the instruction count
of one compression in the compiled gfx950 code of this library (the F step
of a WOTS+ chain, which is over 90 % of all compressions, and the SHA-512
block), counted from its disassembly and confirmed by SQ_INSTS_VALU:
  SHA-256: 1232 (rounds 0-4 of every chain step and 7 of the 48 schedule
           words depend only on the chain's address, so they are computed
           once per chain, not per step);
  SHA-512: 3490 (rounds 0-15 peeled, about 490 instructions, then four
           16-round blocks of about 750; every 64-bit add is one
           v_lshl_add_u64).
SQ_INSTS_VALU of whole launches agrees within 2 % (the rest is loads,
address arithmetic and lanes masked off in the upper Merkle levels).

The SHAKE sets (FIPS 205 Section 11.1) count Keccak-f[1600] permutations
instead: F, PRF and H absorb one 136-byte block, T_l takes
ceil((n + 32 + l n + 1) / 136) blocks, PRF_msg and H_msg absorb their
concatenated inputs.  One permutation on 32-bit lanes (a 64-bit lane as two
halves) is 24 rounds of 180 instructions: theta 20 three-input XORs for
the column parities, 10 alignbits for their 1-bit rotates, 50 three-input
XORs to apply them; rho 48 alignbits (24 rotated lanes); chi 50 one-
instruction a ^ (~b & c); iota 2 XORs.  The compiled round body is exactly
that count (240 v_bitop3 + 116 v_alignbit + 4 v_xor per two rounds).
For comparison, the textbook count with one instruction per primitive of
FIPS 180-4 and no precomputation is:
  SHA-256: round = Sigma1 (3 rotates + 1 xor3) + Ch + Sigma0 (3 + 1) + Maj
           + 4 three-input adds = 14; schedule word = 2 x (2 rotates +
           1 shift + 1 xor3) + 2 adds = 10; feed-forward 8.
           64 * 14 + 48 * 10 + 8 = 1384.
  SHA-512: on 32-bit lanes every 64-bit rotate, xor3, Ch, Maj is 2
           instructions and every 64-bit add 2 (add + carry):
           round = 8 + 8 + 2 + 2 + 7 adds * 2 = 34; schedule word = 8 + 8
           + 3 adds * 2 = 22; feed-forward 16.
           80 * 34 + 64 * 22 + 16 = 4144.
"""
from __future__ import annotations

from dataclasses import dataclass

TEXTBOOK_SHA256 = 64 * 14 + 48 * 10 + 8
TEXTBOOK_SHA512 = 80 * 34 + 64 * 22 + 16
OPS_SHA256 = 1232
OPS_SHA512 = 3490
TEXTBOOK_KECCAK = OPS_KECCAK = 24 * (20 + 10 + 50 + 48 + 50 + 2)

# MI355X VALU issue ceilings for 32-bit integer lane-operations.  A wave64
# instruction occupies a SIMD for 4 clocks at 16 lanes per clock, but on
# gfx950 the simple operations (v_bitop3, v_xor/or/and/not, v_add/sub,
# v_lshrrev, v_mov) issue faster: the valu_probe program measures up to 1.68
# wave64 instructions per 4 SIMD clocks for them, against 0.85-0.95 for
# v_alignbit, v_add3, v_perm, v_lshlrev, v_lshl_add_u64 and the other
# three-operand or 64-bit forms.  The roofline peak is therefore the
# dual-rate ceiling, 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 78.6 T
# lane-ops/s (the same figure as the published FP32 vector rate counted in
# FMA lane-operations).
CUS, SIMDS, LANES, CLOCK_HZ = 256, 4, 16, 2.4e9
VALU_SINGLE_RATE_OPS = CUS * SIMDS * LANES * CLOCK_HZ   # 3.93e13 lane-ops/s
VALU_PEAK_OPS = 2 * VALU_SINGLE_RATE_OPS                 # 7.86e13 lane-ops/s

# Rate each hash's instruction mix reaches with no loads, stores or barriers:
# valu_probe runs the library's own SHA-256 / SHA-512 compressions and
# Keccak-f[1600] on every lane of a full grid (lane-ops/s; SHA-256 1399,
# SHA-512 3417 and Keccak-f 4320 instructions per unit in that program).  The
# rotates are single-rate v_alignbit (41 % of SHA-256, 32 % of Keccak-f), so
# these mixes stay near the single-rate line.
MIX_CEILING_OPS = {"sha256": 39.62e12, "sha512": 39.14e12, "keccak": 42.66e12}


def mix_ceiling_seconds(units: dict) -> float:
    """Shortest time for {hash: units} at the measured mix ceilings."""
    ops = {"sha256": OPS_SHA256, "sha512": OPS_SHA512, "keccak": OPS_KECCAK}
    return sum(units[h] * ops[h] / MIX_CEILING_OPS[h] for h in units)


@dataclass(frozen=True)
class Params:
    n: int
    h: int
    d: int
    a: int
    k: int
    shake: bool = False

    @property
    def hp(self):
        return self.h // self.d

    @property
    def len(self):
        return 2 * self.n + 3

    @property
    def wide(self):
        return self.n >= 24 and not self.shake


PARAMS = {1: Params(16, 66, 22, 6, 33), 2: Params(24, 66, 22, 8, 33), 3: Params(32, 68, 17, 9, 35),
          4: Params(16, 63, 7, 12, 14), 5: Params(24, 63, 7, 14, 17), 6: Params(32, 64, 8, 14, 22)}
PARAMS.update({i + 6: Params(p.n, p.h, p.d, p.a, p.k, True) for i, p in list(PARAMS.items())})


def full_name(param: int) -> str:
    """SHA2-128f ... SHAKE-256s."""
    p = PARAMS[param]
    return "%s-%d%s" % ("SHAKE" if p.shake else "SHA2", 8 * p.n, "s" if p.hp >= 8 else "f")


def t_blocks(p: Params, l: int) -> int:
    """Compressions of T_l after the PK.seed block (SHA2 sets), or Keccak-f
    permutations of T_l (SHAKE sets)."""
    if p.shake:
        return (p.n + 32 + l * p.n + 1 + 135) // 136
    mb = 22 + l * p.n
    if p.wide:
        return (mb + 17 + 127) // 128
    return (mb + 9 + 63) // 64


def per_signature(param: int) -> dict:
    """Compressions (Keccak-f permutations for the SHAKE sets) of one
    signature on the signing path, split by phase and hash (no WOTS+
    recomputation: the chain values are kept)."""
    p = PARAMS[param]
    leaves = p.d << p.hp
    fors_leaves = p.k << p.a
    if p.shake:
        kf = {"fors": 2 * fors_leaves + (fors_leaves - p.k) + t_blocks(p, p.k),
              "tree": leaves * p.len * 16 + leaves * t_blocks(p, p.len) + p.d * ((1 << p.hp) - 1),
              "wots": 0}
        zero = {ph: 0 for ph in kf}
        return {"sha256": zero, "sha512": dict(zero), "keccak": kf}
    c256 = {}
    c512 = {}
    c256["fors"] = 2 * fors_leaves + (0 if p.wide else (fors_leaves - p.k) + t_blocks(p, p.k))
    c512["fors"] = ((fors_leaves - p.k) + t_blocks(p, p.k)) if p.wide else 0
    chains = leaves * p.len * 16
    tlen = leaves * t_blocks(p, p.len)
    merkle = p.d * ((1 << p.hp) - 1)
    c256["tree"] = chains + (0 if p.wide else tlen + merkle)
    c512["tree"] = (tlen + merkle) if p.wide else 0
    c256["wots"] = c512["wots"] = 0
    return {"sha256": c256, "sha512": c512, "keccak": {ph: 0 for ph in c256}}


def prelude_compressions(param: int, mlen: int) -> tuple[int, int]:
    """(SHA-256, SHA-512) compressions of the prelude of one message of mlen
    bytes: R = PRF_msg = HMAC(SK.prf, opt_rand | M) (the inner hash over
    the key block, opt_rand and M; the outer over the key block and the
    inner digest) and H_msg = MGF1(R | PK.seed | Hash(R | PK.seed | PK.root
    | M), m)."""
    p = PARAMS[param]
    m = (p.k * p.a + 7) // 8 + (p.h - p.hp + 7) // 8 + (p.hp + 7) // 8
    if p.shake:
        return 0, 0
    if not p.wide:
        blk = lambda b: (b + 9 + 63) // 64  # noqa: E731
        prf = blk(64 + p.n + mlen) + blk(64 + 32)
        hm = blk(3 * p.n + mlen) + -(-m // 32) * blk(2 * p.n + 32 + 4)
        return prf + hm, 0
    blk = lambda b: (b + 17 + 127) // 128  # noqa: E731
    prf = blk(128 + p.n + mlen) + blk(128 + 64)
    hm = blk(3 * p.n + mlen) + -(-m // 64) * blk(2 * p.n + 64 + 4)
    return 0, prf + hm


def prelude_permutations(param: int, mlen: int) -> int:
    """Keccak-f permutations of the prelude of one message (SHAKE sets):
    PRF_msg = SHAKE256(SK.prf | opt_rand | M, 8n) and
    H_msg = SHAKE256(R | PK.seed | PK.root | M, 8m), m <= 136."""
    p = PARAMS[param]
    if not p.shake:
        return 0
    blk = lambda b: (b + 1 + 135) // 136  # noqa: E731
    return blk(2 * p.n + mlen) + blk(3 * p.n + mlen)


def prelude_ops(param: int, mlen: int) -> int:
    """Textbook VALU operations of the prelude of one message."""
    c256, c512 = prelude_compressions(param, mlen)
    return (c256 * TEXTBOOK_SHA256 + c512 * TEXTBOOK_SHA512
            + prelude_permutations(param, mlen) * TEXTBOOK_KECCAK)


def wots_gather_bytes(param: int) -> int:
    """HBM bytes of the WOTS+ phase per signature when the chain values are
    kept: one n-byte value read and one written per chain of every layer,
    plus the k FORS roots read and the FORS pk written."""
    p = PARAMS[param]
    return 2 * p.d * p.len * p.n + (p.k + 1) * p.n


def ops_per_signature(param: int, phase: str | None = None, textbook: bool = False) -> int:
    """VALU lane-operations per signature (ISA counts, or the textbook counts)."""
    c = per_signature(param)
    o256, o512 = (TEXTBOOK_SHA256, TEXTBOOK_SHA512) if textbook else (OPS_SHA256, OPS_SHA512)
    ok = TEXTBOOK_KECCAK if textbook else OPS_KECCAK
    phases = [phase] if phase else list(c["sha256"])
    return sum(c["sha256"][ph] * o256 + c["sha512"][ph] * o512 + c["keccak"][ph] * ok for ph in phases)


def compressions_per_signature(param: int) -> tuple[int, int]:
    c = per_signature(param)
    return sum(c["sha256"].values()), sum(c["sha512"].values())


def permutations_per_signature(param: int) -> int:
    return sum(per_signature(param)["keccak"].values())
