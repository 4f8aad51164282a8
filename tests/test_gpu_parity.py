"""GPU parity: every signature from the HIP path equals the oracle's, byte
for byte (bit-exact is the only bar: signing is deterministic integer
hashing, so there is exactly one correct signature per key and message).
"""
import os
import sys

import numpy as np
import pytest

import oracle
from helpers import NAMES, describe_diff, oracle_keys, oracle_sign_many
from paper_2512_23969_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2512_23969_amd import slh as m
    return m


@pytest.fixture(scope="module")
def ctx(slh):
    c = slh.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _assert_same(param, got, want, what):
    assert len(got) == len(want)
    for i, (g, w) in enumerate(zip(got, want)):
        assert g == w, "%s item %d: %s" % (what, i, describe_diff(param, g, w))


@pytest.mark.parametrize("param", [1, 2, 3])
def test_keygen_matches_oracle(slh, param):
    for i in range(2):
        seed = workloads.key_seed(param, i)
        _say("keygen", NAMES[param], i)
        assert slh.keygen(param, seed) == oracle.keygen(oracle.params(NAMES[param]), seed)


def test_c1_128f_16_messages(slh, ctx):
    cfg = workloads.CONFIGS["c1_128f_16"]
    seed = workloads.key_seed(1, 0)
    pk, sk = oracle_keys(1, [seed])[0]
    slot = ctx.add_keys(1, sk)
    msgs = workloads.messages(cfg["cfg"], cfg["batch"], cfg["length"])
    _say("sign c1")
    got = slh.sign_messages(ctx, [1] * len(msgs), [slot] * len(msgs), msgs)
    want = oracle_sign_many([(1, sk, m) for m in msgs])
    _assert_same(1, got, want, "c1")
    assert all(oracle.verify(oracle.params("128f"), m, s, pk) for m, s in zip(msgs[:2], got[:2]))


@pytest.mark.parametrize("param", [2, 3])
def test_small_batches_192f_256f(slh, ctx, param):
    seed = workloads.key_seed(param, 0)
    pk, sk = oracle_keys(param, [seed])[0]
    slot = ctx.add_keys(param, sk)
    msgs = workloads.messages(20 + param, 6, 32)
    _say("sign", NAMES[param])
    got = slh.sign_messages(ctx, [param] * len(msgs), [slot] * len(msgs), msgs)
    want = oracle_sign_many([(param, sk, m) for m in msgs])
    _assert_same(param, got, want, NAMES[param])


def test_mixed_batch_lengths_and_keys(slh, ctx):
    """All parameter sets, several keys, message lengths across every SHA-2
    padding edge, in one call; each equals the oracle and its own
    single-request signature."""
    rng = np.random.default_rng([77, 1])
    keys = {}
    for param in (1, 2, 3):
        for i in range(2):
            seed = workloads.key_seed(param, 10 + i)
            pk, sk = oracle_keys(param, [seed])[0]
            keys[(param, i)] = (ctx.add_keys(param, sk), sk, pk)
    lengths = [0, 1, 3, 31, 55, 56, 63, 64, 65, 111, 112, 119, 127, 128, 129, 300, 1000, 4099]
    jobs, params, slots, msgs = [], [], [], []
    for j, L in enumerate(lengths):
        param = 1 + j % 3
        slot, sk, pk = keys[(param, j % 2)]
        m = rng.bytes(L)
        params.append(param); slots.append(slot); msgs.append(m); jobs.append((param, sk, m))
    _say("sign mixed")
    got = slh.sign_messages(ctx, params, slots, msgs)
    want = oracle_sign_many(jobs)
    for i in range(len(msgs)):
        assert got[i] == want[i], "len %d %s: %s" % (len(msgs[i]), NAMES[params[i]],
                                                     describe_diff(params[i], got[i], want[i]))
    # the same request alone gives the same bytes
    alone = slh.sign_messages(ctx, params[5:6], slots[5:6], msgs[5:6])
    assert alone[0] == got[5]


@pytest.mark.parametrize("param", [1, 3, 7, 9])
def test_unaligned_message_offsets(slh, ctx, param):
    seed = workloads.key_seed(param, 3)
    pk, sk = oracle_keys(param, [seed])[0]
    slot = ctx.add_keys(param, sk)
    import torch
    blob = bytes(range(256)) * 8
    # odd and aligned offsets; long messages cover whole blocks read byte by
    # byte (odd offsets) and as aligned dwords (offsets 4 and 1032)
    offs = [1, 7, 130, 333, 999, 3, 4, 1032, 1]
    lens = [5, 60, 1, 200, 25, 600, 700, 513, 2047]
    n = len(offs)
    items = np.zeros(n, dtype=slh.ITEM_DTYPE)
    sigb = slh.sizes(param)["sig_bytes"]
    for i in range(n):
        items[i] = (param, slot, offs[i], lens[i], i * sigb)
    d_m = torch.frombuffer(bytearray(blob), dtype=torch.uint8).cuda()
    d_s = torch.zeros(n * sigb, dtype=torch.uint8, device="cuda")
    ctx.sign_batch(items, d_m, d_s)
    torch.cuda.synchronize()
    host = d_s.cpu().numpy().tobytes()
    want = oracle_sign_many([(param, sk, blob[o:o + L]) for o, L in zip(offs, lens)])
    for i in range(n):
        assert host[i * sigb:(i + 1) * sigb] == want[i], "offset %d length %d" % (offs[i], lens[i])


@pytest.mark.parametrize("param", [1, 2, 3])
def test_gpu_verify(slh, param):
    seed = workloads.key_seed(param, 0)
    pk, sk = oracle_keys(param, [seed])[0]
    p = oracle.params(NAMES[param])
    msg = b"verify me"
    sig = oracle.sign(p, msg, sk)
    assert slh.verify(param, msg, sig, pk)
    for off in (0, p.n, len(sig) // 2, len(sig) - 1):
        bad = bytearray(sig)
        bad[off] ^= 4
        assert not slh.verify(param, msg, bytes(bad), pk)
    assert not slh.verify(param, msg + b".", sig, pk)
    assert not slh.verify(param, msg, sig[:-1], pk)


def test_invalid_arguments(slh, ctx):
    import torch
    seed = workloads.key_seed(1, 0)
    pk, sk = oracle_keys(1, [seed])[0]
    slot = ctx.add_keys(1, sk)
    sigb = slh.sizes(1)["sig_bytes"]
    d_m = torch.zeros(64, dtype=torch.uint8, device="cuda")
    d_s = torch.full((2 * sigb,), 7, dtype=torch.uint8, device="cuda")
    cases = {
        "bad slot": [(1, 10 ** 6, 0, 4, 0)],
        "param mismatch": [(2, slot, 0, 4, 0)],
        "msg out of range": [(1, slot, 60, 8, 0)],
        "sig out of range": [(1, slot, 0, 4, sigb + 16)],
        "sig misaligned": [(1, slot, 0, 4, 8)],
        "overlap": [(1, slot, 0, 4, 0), (1, slot, 0, 4, 16)],
        "bad param": [(13, slot, 0, 4, 0)],
        "param zero": [(0, slot, 0, 4, 0)],
        "set of another shape": [(5, slot, 0, 4, 0)],
        "same shape, other hash": [(7, slot, 0, 4, 0)],
    }
    for name, rows in cases.items():
        items = np.array(rows, dtype=slh.ITEM_DTYPE)
        with pytest.raises(slh.SlhError) as e:
            ctx.sign_batch(items, d_m, d_s)
        assert e.value.code == slh.EINVAL, name
    torch.cuda.synchronize()
    assert bool((d_s == 7).all()), "nothing may be written on EINVAL"
    with pytest.raises(slh.SlhError):
        ctx.sign_batch(np.array([(1, slot, 0, 4, 0)], dtype=slh.ITEM_DTYPE), d_m, d_s, mode=99)


def test_empty_batches(slh, ctx):
    """Zero requests: signing, verification and the external interface
    return OK and write nothing."""
    import torch
    d_m = torch.zeros(16, dtype=torch.uint8, device="cuda")
    d_s = torch.full((64,), 5, dtype=torch.uint8, device="cuda")
    for mode in ("plain", "fused", "graph-dedup"):
        ctx.sign_batch(np.zeros(0, dtype=slh.ITEM_DTYPE), d_m, d_s, mode=slh.MODES[mode])
    ctx.sign_batch_ext(np.zeros(0, dtype=slh.ITEM_EXT_DTYPE), d_m, d_s)
    res = torch.full((4,), -1, dtype=torch.int32, device="cuda")
    ctx.verify_batch(np.zeros(0, dtype=slh.VERIFY_DTYPE), d_m, d_s, d_m, res)
    torch.cuda.synchronize()
    assert bool((d_s == 5).all()) and bool((res == -1).all())


def test_repeat_determinism(slh, ctx):
    seed = workloads.key_seed(3, 5)
    pk, sk = oracle_keys(3, [seed])[0]
    slot = ctx.add_keys(3, sk)
    msgs = workloads.messages(31, 40, 32)
    a = slh.sign_messages(ctx, [3] * 40, [slot] * 40, msgs)
    b = slh.sign_messages(ctx, [3] * 40, [slot] * 40, msgs)
    assert a == b
    want = oracle_sign_many([(3, sk, msgs[0]), (3, sk, msgs[-1])])
    assert a[0] == want[0] and a[-1] == want[1]


def test_small_memory_budget_chunks(slh):
    """A context with a budget of a few messages processes a batch in chunks."""
    seed = workloads.key_seed(2, 6)
    pk, sk = oracle_keys(2, [seed])[0]
    c = slh.Context(0, hbm_budget=3 * 1024 * 1024)
    try:
        slot = c.add_keys(2, sk)
        msgs = workloads.messages(41, 9, 32)
        got = slh.sign_messages(c, [2] * 9, [slot] * 9, msgs)
    finally:
        c.close()
    want = oracle_sign_many([(2, sk, m) for m in msgs])
    _assert_same(2, got, want, "chunked")
