"""The work accounting used by the benchmark's roofline agrees with the
oracle's own hash-block counters and with the paper's printed counts."""
import json
import os

import pytest

import oracle
from paper_2512_23969_amd import accounting as acc

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_figures.json")))
NAMES = {1: "128f", 2: "192f", 3: "256f"}


@pytest.mark.parametrize("param", [1, 2, 3])
def test_compressions_per_signature(param):
    # exact totals of the signing path without WOTS+ recomputation
    want = {1: (106786, 0), 2: (160512, 10336), 3: (327424, 23046)}[param]
    assert acc.compressions_per_signature(param) == want


@pytest.mark.parametrize("param", [1, 2, 3])
def test_chain_hashes_per_leaf_match_paper(param):
    p = acc.PARAMS[param]
    assert p.len * 16 == GOLD["hashes_per_wots_leaf"][NAMES[param]]


@pytest.mark.parametrize("param", [1, 2, 3])
def test_t_blocks_match_oracle_block_counter(param):
    """T_len and T_k compressions counted by the oracle's SHA-2 block counters
    (each tweakable hash also compresses the PK.seed block first)."""
    p = oracle.params(NAMES[param])
    a = acc.PARAMS[param]
    for l in (p.len, p.k, 2):
        oracle.counters_reset()
        oracle.T(p, bytes(p.n), bytes(32), bytes(l * p.n))
        c = oracle.counters()
        blocks = c["sha512_blocks"] if p.wide else c["sha256_blocks"]
        assert blocks - 1 == acc.t_blocks(a, l)


def test_isa_costs_below_textbook():
    assert acc.OPS_SHA256 < acc.TEXTBOOK_SHA256 == 1384
    assert acc.OPS_SHA512 > acc.TEXTBOOK_SHA512 * 0 and acc.TEXTBOOK_SHA512 == 4144
    assert abs(acc.VALU_SINGLE_RATE_OPS - 39.3216e12) < 1e9
    assert abs(acc.VALU_PEAK_OPS - 78.6432e12) < 1e9
    # the measured mix ceilings lie between the single-rate and dual-rate lines
    for v in acc.MIX_CEILING_OPS.values():
        assert acc.VALU_SINGLE_RATE_OPS * 0.95 < v < acc.VALU_PEAK_OPS


@pytest.mark.parametrize("param", [1, 2, 3])
@pytest.mark.parametrize("mlen", [0, 32, 55, 56, 200, 1000])
def test_prelude_compressions_match_oracle(param, mlen):
    """PRF_msg + H_msg block counts (the prelude's roofline units) equal the
    oracle's SHA-2 block counters."""
    p = oracle.params(NAMES[param])
    n = p.n
    oracle.counters_reset()
    r = oracle.prf_msg(p, bytes(n), bytes(n), bytes(mlen))
    oracle.h_msg(p, r, bytes(n), bytes(n), bytes(mlen))
    c = oracle.counters()
    assert (c["sha256_blocks"], c["sha512_blocks"]) == acc.prelude_compressions(param, mlen)


SHAKE_NAMES = {7: "shake-128f", 8: "shake-192f", 9: "shake-256f", 10: "shake-128s", 11: "shake-192s",
               12: "shake-256s"}


@pytest.mark.parametrize("param", sorted(SHAKE_NAMES))
def test_shake_t_permutations_match_oracle(param):
    """Keccak-f permutations of T_l (SHAKE sets) equal the oracle's
    permutation counter; F/H take one."""
    p = oracle.params(SHAKE_NAMES[param])
    a = acc.PARAMS[param]
    for l in (p.len, p.k, 2, 1):
        oracle.counters_reset()
        oracle.T(p, bytes(p.n), bytes(32), bytes(l * p.n))
        want = acc.t_blocks(a, l) if l > 2 else 1
        assert oracle.counters()["keccak_f"] == want


@pytest.mark.parametrize("param", [7, 9, 11])
@pytest.mark.parametrize("mlen", [0, 32, 40, 88, 89, 200, 1000])
def test_prelude_permutations_match_oracle(param, mlen):
    p = oracle.params(SHAKE_NAMES[param])
    n = p.n
    oracle.counters_reset()
    r = oracle.prf_msg(p, bytes(n), bytes(n), bytes(mlen))
    oracle.h_msg(p, r, bytes(n), bytes(n), bytes(mlen))
    c = oracle.counters()
    assert c["keccak_f"] == acc.prelude_permutations(param, mlen)
    assert (c["sha256_blocks"], c["sha512_blocks"]) == acc.prelude_compressions(param, mlen) == (0, 0)


def test_keccak_round_cost():
    # theta 20 + 10 + 50, rho 48, chi 50, iota 2 per round
    assert acc.OPS_KECCAK == acc.TEXTBOOK_KECCAK == 24 * 180


@pytest.mark.parametrize("sp", [1, 2, 3, 4, 5, 6])
def test_shake_sets_hash_the_same_trees(sp):
    """Apart from the blocks of T_l, a SHAKE set makes one permutation per
    tweakable-hash call where its SHA2 twin makes one compression."""
    a, b = acc.PARAMS[sp], acc.PARAMS[sp + 6]
    s, k = acc.per_signature(sp), acc.per_signature(sp + 6)
    leaves = a.d << a.hp
    sha_tree = s["sha256"]["tree"] + s["sha512"]["tree"] - leaves * acc.t_blocks(a, a.len)
    assert k["keccak"]["tree"] - leaves * acc.t_blocks(b, b.len) == sha_tree
    sha_fors = s["sha256"]["fors"] + s["sha512"]["fors"] - acc.t_blocks(a, a.k)
    assert k["keccak"]["fors"] - acc.t_blocks(b, b.k) == sha_fors == 3 * (a.k << a.a) - a.k
