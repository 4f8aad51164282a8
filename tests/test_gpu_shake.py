"""GPU parity of the SHAKE256 instantiation (FIPS 205 Section 11.1) for the
six shapes: SHAKE-128f/192f/256f (ids 7-9, every signing mode: per-phase,
fused, dedup, graph) and SHAKE-128s/192s/256s (ids 10-12, unit-built trees).
Keys, signatures and GPU verification must match the oracle byte for byte;
the message lengths straddle the 136-byte SHAKE256 rate once the 2n-byte
(PRF_msg) and 3n-byte (H_msg) prefixes are counted."""
import numpy as np
import pytest

import oracle
from helpers import NAMES, describe_diff, oracle_keys, oracle_sign_many
from paper_2512_23969_amd import workloads

pytestmark = pytest.mark.gpu
FAST = (7, 8, 9)
SMALL = (10, 11, 12)


@pytest.fixture(scope="module")
def slh():
    import torch
    assert torch.cuda.is_available()
    from paper_2512_23969_amd import slh as m
    return m


@pytest.fixture(scope="module")
def keys():
    return {p: oracle_keys(p, [workloads.key_seed(p, 900)])[0] for p in FAST + SMALL}


def _lengths(param):
    n = workloads.N_OF[param]
    # total absorbed bytes 135, 136 and 137 after the PRF_msg / H_msg prefixes
    near = sorted({136 - 2 * n - 1, 136 - 2 * n, 136 - 3 * n, 136 - 3 * n + 1, 272 - 3 * n})
    return [0, 1] + near + [1000]


def _gpu_verify(slh, param, pk, msgs, sigs, flip):
    """Verify (msgs[i], sigs[i]) on the GPU plus one copy of the last pair
    with byte `flip` of its signature changed; returns the result list."""
    import torch
    sb = slh.sizes(param)["sig_bytes"]
    vit = np.zeros(len(msgs) + 1, dtype=slh.VERIFY_DTYPE)
    off = 0
    for i, m in enumerate(msgs):
        vit[i] = (param, 0, off, len(m), i * sb, 0)
        off += len(m)
    bad = bytearray(sigs[-1])
    bad[flip] ^= 0x10
    vit[len(msgs)] = (param, 0, off - len(msgs[-1]), len(msgs[-1]), len(msgs) * sb, 0)
    d_m = torch.frombuffer(bytearray(b"".join(msgs) + b"\0"), dtype=torch.uint8).cuda()
    d_s = torch.frombuffer(bytearray(b"".join(sigs) + bytes(bad)), dtype=torch.uint8).cuda()
    d_pk = torch.frombuffer(bytearray(pk), dtype=torch.uint8).cuda()
    res = torch.full((len(msgs) + 1,), -1, dtype=torch.int32, device="cuda")
    with slh.Context(0) as ctx:
        ctx.verify_batch(vit, d_m, d_s, d_pk, res)
        torch.cuda.synchronize()
    return res.cpu().tolist()


@pytest.mark.parametrize("param", FAST + SMALL)
def test_shake_keygen(slh, keys, param):
    print("keygen", NAMES[param], flush=True)
    assert slh.keygen(param, workloads.key_seed(param, 900)) == keys[param]


@pytest.mark.parametrize("param", FAST)
def test_shake_fast_sign_matches_oracle(slh, keys, param):
    pk, sk = keys[param]
    rng = np.random.default_rng([61, param])
    msgs = [rng.bytes(L) for L in _lengths(param)]
    want = oracle_sign_many([(param, sk, m) for m in msgs])
    with slh.Context(0) as ctx:
        slot = ctx.add_keys(param, sk)
        for mode in ("plain", "fused", "dedup", "graph-dedup", "fused-dedup"):
            print(NAMES[param], mode, flush=True)
            got = slh.sign_messages(ctx, [param] * len(msgs), [slot] * len(msgs), msgs, slh.MODES[mode])
            for i, (g, w) in enumerate(zip(got, want)):
                assert g == w, "%s msg %d B: %s" % (mode, len(msgs[i]), describe_diff(param, g, w))
        # the tree cache of the fast sets (read by the dedup modes)
        ctx.cache_keys(slot, 1, 2)
        for mode in ("dedup", "fused-dedup"):
            print(NAMES[param], "cached", mode, flush=True)
            got = slh.sign_messages(ctx, [param] * len(msgs), [slot] * len(msgs), msgs, slh.MODES[mode])
            assert got == want
    sb = slh.sizes(param)["sig_bytes"]
    assert _gpu_verify(slh, param, pk, msgs, want, sb // 2) == [1] * len(msgs) + [0]


@pytest.mark.parametrize("param", SMALL)
def test_shake_small_sign_matches_oracle(slh, keys, param):
    pk, sk = keys[param]
    rng = np.random.default_rng([67, param])
    msgs = [rng.bytes(L) for L in (0, 136 - 3 * workloads.N_OF[param], 500)]
    want = oracle_sign_many([(param, sk, m) for m in msgs])
    with slh.Context(0) as ctx:
        slot = ctx.add_keys(param, sk)
        for mode in ("plain", "graph-dedup"):
            print(NAMES[param], mode, flush=True)
            got = slh.sign_messages(ctx, [param] * len(msgs), [slot] * len(msgs), msgs, slh.MODES[mode])
            for i, (g, w) in enumerate(zip(got, want)):
                assert g == w, "%s msg %d B: %s" % (mode, len(msgs[i]), describe_diff(param, g, w))
        with pytest.raises(slh.SlhError):
            ctx.cache_keys(slot, 1, 1)
    sb = slh.sizes(param)["sig_bytes"]
    assert _gpu_verify(slh, param, pk, msgs, want, sb - 3) == [1] * len(msgs) + [0]


def test_shake_and_sha2_in_one_batch(slh, keys):
    """A batch mixing SHA2 and SHAKE keys of equal shape: each request is
    hashed with its own instantiation."""
    sha = {p: oracle_keys(p, [workloads.key_seed(p, 901)])[0] for p in (1, 3, 4)}
    allk = {**keys, **sha}
    rng = np.random.default_rng(71)
    params = [7, 1, 9, 3, 10, 4, 8, 7, 1]
    msgs = [rng.bytes(int(rng.integers(0, 200))) for _ in params]
    want = oracle_sign_many([(p, allk[p][1], m) for p, m in zip(params, msgs)])
    with slh.Context(0) as ctx:
        slots = {p: ctx.add_keys(p, allk[p][1]) for p in sorted(set(params))}
        for mode in ("fused-dedup", "plain"):
            print("mixed", mode, flush=True)
            got = slh.sign_messages(ctx, params, [slots[p] for p in params], msgs, slh.MODES[mode])
            for i, p in enumerate(params):
                assert got[i] == want[i], "%s item %d (%s): %s" % (mode, i, NAMES[p],
                                                                   describe_diff(p, got[i], want[i]))


def test_shake_ext_interface(slh, keys):
    """Pure and HashSLH-DSA signing with context strings and hedged
    randomness on a SHAKE key (FIPS 205 Algorithms 22-23)."""
    param = 7
    pk, sk = keys[param]
    p = oracle.params(NAMES[param])
    rng = np.random.default_rng(73)
    cases = [(rng.bytes(ml), c, ph, rng.bytes(16) if h else None)
             for ml, c, ph, h in ((0, b"", 0, False), (100, b"ctx", 0, True), (300, b"x" * 200, 1, False),
                                  (33, b"", 2, True))]
    want = [oracle.sign_ext(p, m, sk, c, ph, r) for m, c, ph, r in cases]
    with slh.Context(0) as ctx:
        slot = ctx.add_keys(param, sk)
        for mode in ("plain", "fused"):
            print("ext", mode, flush=True)
            got = slh.sign_messages_ext(ctx, [param] * len(cases), [slot] * len(cases), [c[0] for c in cases],
                                        [c[1] for c in cases], [c[2] for c in cases], [c[3] for c in cases],
                                        slh.MODES[mode])
            assert got == want
    for g, (m, c, ph, _) in zip(want, cases):
        assert oracle.verify_ext(p, m, g, pk, c, ph)
