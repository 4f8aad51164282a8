"""GPU parity of the SHA2 small parameter sets (128s, 192s, 256s; FIPS 205
Table 2).  Their XMSS trees (2^8-2^9 leaves) and FORS trees (2^12-2^14
leaves) are built in units of 64 and 2^12 leaves whose roots a combine step
joins; keys, signatures (in every mode flag, which these sets take through
the per-phase path) and GPU verification must match the oracle."""
import numpy as np
import pytest

import oracle
from helpers import NAMES, describe_diff, oracle_keys, oracle_sign_many
from paper_2512_23969_amd import workloads

pytestmark = pytest.mark.gpu
SMALL = (4, 5, 6)


@pytest.fixture(scope="module")
def slh():
    import torch
    assert torch.cuda.is_available()
    from paper_2512_23969_amd import slh as m
    return m


@pytest.fixture(scope="module")
def keys():
    return {p: oracle_keys(p, [workloads.key_seed(p, 800)])[0] for p in SMALL}


@pytest.mark.parametrize("param", SMALL)
def test_small_keygen(slh, keys, param):
    pk, sk = keys[param]
    gpk, gsk = slh.keygen(param, workloads.key_seed(param, 800))
    assert (gpk, gsk) == (pk, sk)


@pytest.mark.parametrize("param", SMALL)
def test_small_sign_matches_oracle(slh, keys, param):
    import torch
    pk, sk = keys[param]
    rng = np.random.default_rng([51, param])
    msgs = [rng.bytes(L) for L in (0, 1, 33, 200, 1000)]
    want = oracle_sign_many([(param, sk, m) for m in msgs])
    with slh.Context(0) as ctx:
        slot = ctx.add_keys(param, sk)
        for mode in ("plain", "graph-dedup"):
            print(NAMES[param], mode, flush=True)
            got = slh.sign_messages(ctx, [param] * len(msgs), [slot] * len(msgs), msgs, slh.MODES[mode])
            for i, (g, w) in enumerate(zip(got, want)):
                assert g == w, "%s item %d: %s" % (mode, i, describe_diff(param, g, w))
        for fg, keep in ((2, 1), (1, 0)):
            ctx.set_tuning(param, fg, 0, keep)
            print(NAMES[param], "fg", fg, "keep", keep, flush=True)
            got = slh.sign_messages(ctx, [param] * 2, [slot] * 2, msgs[2:4])
            assert got == want[2:4]
        with pytest.raises(slh.SlhError):
            ctx.cache_keys(slot, 1, 1)
        # GPU verification: all accepted, a flipped byte rejected
        blob = b"".join(msgs)
        sb = slh.sizes(param)["sig_bytes"]
        vit = np.zeros(len(msgs) + 1, dtype=slh.VERIFY_DTYPE)
        off = 0
        for i, m in enumerate(msgs):
            vit[i] = (param, 0, off, len(m), i * sb, 0)
            off += len(m)
        bad = bytearray(want[4])
        bad[sb // 3] ^= 4
        vit[len(msgs)] = (param, 0, off - len(msgs[4]), len(msgs[4]), len(msgs) * sb, 0)
        d_m = torch.frombuffer(bytearray(blob), dtype=torch.uint8).cuda()
        d_s = torch.frombuffer(bytearray(b"".join(want) + bytes(bad)), dtype=torch.uint8).cuda()
        d_pk = torch.frombuffer(bytearray(pk), dtype=torch.uint8).cuda()
        res = torch.full((len(msgs) + 1,), -1, dtype=torch.int32, device="cuda")
        ctx.verify_batch(vit, d_m, d_s, d_pk, res)
        torch.cuda.synchronize()
        assert res.cpu().tolist() == [1] * len(msgs) + [0]


def test_small_and_fast_sets_in_one_batch(slh, keys):
    """One call mixing all six sets, in the fused-dedup mode (the fast sets
    take the fused and dedup paths, the small sets the per-phase one)."""
    fast = {p: oracle_keys(p, [workloads.key_seed(p, 801)])[0] for p in (1, 2, 3)}
    allk = {**keys, **fast}
    rng = np.random.default_rng(53)
    params = [4, 1, 5, 2, 6, 3, 4, 1]
    msgs = [rng.bytes(int(rng.integers(0, 120))) for _ in params]
    want = oracle_sign_many([(p, allk[p][1], m) for p, m in zip(params, msgs)])
    with slh.Context(0) as ctx:
        slots = {p: ctx.add_keys(p, allk[p][1]) for p in (1, 2, 3, 4, 5, 6)}
        for mode in ("fused-dedup", "plain"):
            print("mixed", mode, flush=True)
            got = slh.sign_messages(ctx, params, [slots[p] for p in params], msgs, slh.MODES[mode])
            for i, p in enumerate(params):
                assert got[i] == want[i], "%s item %d (%s): %s" % (mode, i, NAMES[p], describe_diff(p, got[i], want[i]))
