"""GPU parity of the batched execution modes and of every tuning knob: the
fused persistent kernel, the captured hipGraph (replayed several times with
new message contents, eager work in between), mixed parameter sets in one
launch, every compiled FORS group size and the recompute-WOTS variant all
give the oracle's signature, byte for byte."""
import numpy as np
import pytest

import oracle
from helpers import NAMES, describe_diff, oracle_keys, oracle_sign_many
from paper_2512_23969_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slh():
    import torch
    assert torch.cuda.is_available()
    from paper_2512_23969_amd import slh as m
    return m


@pytest.fixture(scope="module")
def keys():
    out = {}
    for p in (1, 2, 3):
        seed = workloads.key_seed(p, 20)
        out[p] = oracle_keys(p, [seed])[0]
    return out


def _check(param, got, want, what):
    for i, (g, w) in enumerate(zip(got, want)):
        assert g == w, "%s item %d: %s" % (what, i, describe_diff(param, g, w))


@pytest.mark.parametrize("split", [0, "never"])
@pytest.mark.parametrize("mode", ["fused", "graph", "graph-plain"])
def test_modes_single_set(slh, keys, mode, split):
    """Small batches take the split per-phase path by default; with the split
    off they run the requested kernels (the fused one in fused modes)."""
    with slh.Context(0) as ctx:
        for p in (1, 2, 3):
            pk, sk = keys[p]
            slot = ctx.add_keys(p, sk)
            if split == "never":
                ctx.set_tuning(p, split_max_blocks=slh.SPLIT_NEVER)
            msgs = workloads.messages(60 + p, 5 + p, 32)
            print(mode, NAMES[p], flush=True)
            got = slh.sign_messages(ctx, [p] * len(msgs), [slot] * len(msgs), msgs, slh.MODES[mode])
            _check(p, got, oracle_sign_many([(p, sk, m) for m in msgs]), mode)


def test_graph_mixed_batch_replays(slh, keys):
    """One captured graph with three parameter-set branches, replayed with new
    message bytes of the same layout; every replay matches the oracle."""
    import torch
    rng = np.random.default_rng([61, 0])
    with slh.Context(0) as ctx:
        slots = {p: ctx.add_keys(p, keys[p][1]) for p in (1, 2, 3)}
        params = [1, 2, 3, 1, 3, 2, 1]
        lens = [32, 200, 5, 64, 1000, 0, 33]
        msgs = [rng.bytes(L) for L in lens]
        items, blob, total = slh.pack_batch(params, [slots[p] for p in params], msgs)
        d_m = torch.zeros(max(1, len(blob)), dtype=torch.uint8, device="cuda")
        d_s = torch.zeros(total, dtype=torch.uint8, device="cuda")
        for rep in range(3):
            msgs = [rng.bytes(L) for L in lens]
            _, blob2, _ = slh.pack_batch(params, [slots[p] for p in params], msgs)
            assert len(blob2) == len(blob)
            d_m.copy_(torch.frombuffer(bytearray(blob2 or b"\0"), dtype=torch.uint8))
            print("graph replay", rep, flush=True)
            ctx.sign_batch(items, (d_m.data_ptr(), len(blob)), d_s, slh.MODES["graph"])
            torch.cuda.synchronize()
            host = d_s.cpu().numpy().tobytes()
            got = [host[int(it["sig_off"]):int(it["sig_off"]) + slh.sizes(int(it["param"]))["sig_bytes"]]
                   for it in items]
            want = oracle_sign_many([(p, keys[p][1], m) for p, m in zip(params, msgs)])
            for i, p in enumerate(params):
                assert got[i] == want[i], "replay %d item %d: %s" % (rep, i, describe_diff(p, got[i], want[i]))
            d_s.zero_()  # eager work between replays
            torch.cuda.synchronize()


@pytest.mark.parametrize("param", [1, 2, 3])
def test_every_tuning_variant(slh, keys, param):
    pk, sk = keys[param]
    msgs = workloads.messages(70 + param, 7, 32)
    want = oracle_sign_many([(param, sk, m) for m in msgs])
    with slh.Context(0) as ctx:
        slot = ctx.add_keys(param, sk)
        for fg in slh.FORS_GROUPS[param]:
            for keep in (1, 0):
                for wpc, split in ((0, slh.SPLIT_NEVER), (1, slh.SPLIT_NEVER), (0, 0), (0, 1)):
                    ctx.set_tuning(param, fg, wpc, keep, split)
                    assert ctx.get_tuning(param) == {"fors_trees_per_group": fg, "wgs_per_cu": wpc,
                                                     "keep_chains": keep, "split_max_blocks": split}
                    for mode in ("plain", "fused"):
                        print(NAMES[param], fg, keep, wpc, split, mode, flush=True)
                        got = slh.sign_messages(ctx, [param] * 7, [slot] * 7, msgs, slh.MODES[mode])
                        _check(param, got, want, "fg%d keep%d wpc%d split%d %s" % (fg, keep, wpc, split, mode))


def test_tuning_rejects_uncompiled_variants(slh):
    with slh.Context(0) as ctx:
        with pytest.raises(slh.SlhError):
            ctx.set_tuning(1, 3, 0, 1)
        with pytest.raises(slh.SlhError):
            ctx.set_tuning(3, 16, 0, 1)
        with pytest.raises(slh.SlhError):
            ctx.set_tuning(2, 8, 0, 2)


def test_reserve_then_sign(slh, keys):
    """Working memory reserved up front for the largest batch; smaller and
    mixed batches afterwards still match the oracle."""
    with slh.Context(0, hbm_budget=1 << 30) as ctx:
        slots = {p: ctx.add_keys(p, keys[p][1]) for p in (1, 2, 3)}
        mode = slh.MODES["fused-dedup"]
        ctx.reserve(24, mode)
        rng = np.random.default_rng(77)
        for count in (1, 9, 24):
            params = [(1, 2, 3)[i % 3] for i in range(count)]
            msgs = [rng.bytes(int(rng.integers(0, 90))) for _ in range(count)]
            print("reserve", count, flush=True)
            got = slh.sign_messages(ctx, params, [slots[p] for p in params], msgs, mode)
            want = oracle_sign_many([(p, keys[p][1], m) for p, m in zip(params, msgs)])
            for i, p in enumerate(params):
                assert got[i] == want[i], "count %d item %d: %s" % (count, i, describe_diff(p, got[i], want[i]))
        with pytest.raises(slh.SlhError):
            ctx.reserve(8, 64)


def test_graph_after_key_table_grows(slh, keys):
    """Adding keys can move the device key table; a batch signed in graph mode
    before and after that (same items, same buffers) still matches the oracle,
    so no captured graph keeps the old table's address."""
    import torch
    p = 1
    sk = keys[p][1]
    with slh.Context(0) as ctx:
        slot0 = ctx.add_keys(p, sk)
        msgs = workloads.messages(90, 5, 32)
        want = oracle_sign_many([(p, sk, m) for m in msgs])
        for grow in (0, 1, 2):
            if grow:
                # 100 copies of the key: the table (64 slots at first) is reallocated
                first = ctx.add_keys(p, b"".join([sk] * 100))
                slot = first + 99
            else:
                slot = slot0
            items, blob, total = slh.pack_batch([p] * 5, [slot] * 5, msgs)
            d_m = torch.frombuffer(bytearray(blob), dtype=torch.uint8).cuda()
            d_s = torch.zeros(total, dtype=torch.uint8, device="cuda")
            for rep in range(2):
                print("graph after growth", grow, rep, flush=True)
                ctx.sign_batch(items, (d_m.data_ptr(), len(blob)), d_s, slh.MODES["graph"])
                torch.cuda.synchronize()
                host = d_s.cpu().numpy().tobytes()
                sb = slh.sizes(p)["sig_bytes"]
                for i, it in enumerate(items):
                    o = int(it["sig_off"])
                    assert host[o:o + sb] == want[i], "growth %d replay %d item %d" % (grow, rep, i)
                d_s.zero_()
                torch.cuda.synchronize()
