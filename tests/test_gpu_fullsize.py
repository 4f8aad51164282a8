"""Full-size parity in the launch configurations the benchmark times: each
batch-4096 workload (128f 1 key, 192f 1 key, 256f 64 keys, and the SHAKE
fast sets alike) and each batch-1024 small-set workload, signed in the mode
the benchmark times it in (with that mode's tuned knobs) and in every other
mode (within-batch tree dedup included), gives identical bytes.  Every key
is the oracle's, derived from its seed, and the GPU's key generation must
give the same key for every seed used.  For
the SHA2 fast sets (128f, 192f, 256f over 64 keys) all 4096 signatures equal
the oracle's; for the others a sample (16 plus the first and last) does.
Every signature of the batch verifies on the GPU (a property that holds at
any size), while corrupted copies do not."""
import numpy as np
import pytest

import oracle
from helpers import NAMES, assert_gpu_keys, describe_diff, oracle_keys, oracle_sign_many
from paper_2512_23969_amd import workloads

# workloads whose whole batch is compared with the oracle
FULL_ORACLE = ("c2_128f_4096", "c3_192f_4096", "c4_256f_4096x64")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slh():
    import torch
    assert torch.cuda.is_available()
    from paper_2512_23969_amd import slh as m
    return m


@pytest.mark.parametrize("name", ["c2_128f_4096", "c3_192f_4096", "c4_256f_4096x64", "s1_128s_1024",
                                  "s2_192s_1024", "s3_256s_1024", "k1_shake128f_4096", "k2_shake192f_4096",
                                  "k3_shake256f_4096x64", "k4_shake128s_1024"])
def test_full_batch(slh, name):
    import torch
    from paper_2512_23969_amd import autotune
    cfg = workloads.CONFIGS[name]
    param, batch = cfg["param"], cfg["batch"]
    seeds = [workloads.key_seed(param, i) for i in range(cfg["keys"])]
    keys = oracle_keys(param, seeds)
    assert_gpu_keys(slh, param, seeds, keys)
    kidx = workloads.key_assignment(cfg["cfg"], batch, cfg["keys"]) if cfg["keys"] > 1 else [0] * batch
    msgs = workloads.messages(cfg["cfg"], batch, cfg["length"])
    with slh.Context(0) as ctx:
        first = ctx.add_keys(param, [sk for _, sk in keys])
        slots = [first + k for k in kidx]
        items, blob, total = slh.pack_batch([param] * batch, slots, msgs)
        d_m = torch.frombuffer(bytearray(blob), dtype=torch.uint8).cuda()
        outs = {}
        # the mode and knobs the benchmark times this workload with
        tuned_mode, knobs = autotune.resolve_mode(param, batch, cfg.get("mode", "auto"))
        if knobs:
            autotune.apply(ctx, param, knobs)
        modes = ("plain", "fused", "graph-plain", "graph", "dedup", "fused-dedup", "graph-dedup")
        assert tuned_mode in modes, tuned_mode
        for mode in modes:
            d_s = torch.zeros(total, dtype=torch.uint8, device="cuda")
            print(name, mode, flush=True)
            ctx.sign_batch(items, d_m, d_s, mode=slh.MODES[mode])
            torch.cuda.synchronize()
            outs[mode] = d_s
        for mode in modes[1:]:
            assert torch.equal(outs[mode], outs["plain"]), mode
        # the oracle against the output of the mode the benchmark times
        host = outs[tuned_mode].cpu().numpy().tobytes()
        sb = slh.sizes(param)["sig_bytes"]
        sig = lambda i: host[int(items[i]["sig_off"]):int(items[i]["sig_off"]) + sb]  # noqa: E731
        if name in FULL_ORACLE:
            sample = list(range(batch))
        else:
            sample = workloads.sample_indices(cfg["cfg"], batch, 16)
        print(name, "oracle on", len(sample), "signatures", flush=True)
        want = oracle_sign_many([(param, keys[kidx[i]][1], msgs[i]) for i in sample])
        bad = [i for i, w in zip(sample, want) if sig(i) != w]
        assert not bad, "%s: %d of %d signatures differ from the oracle, first item %d: %s" % (
            name, len(bad), len(sample), bad[0], describe_diff(param, sig(bad[0]), want[sample.index(bad[0])]))
        # every signature verifies on the GPU; flipped copies of a few do not
        pks = b"".join(pk for pk, _ in keys)
        d_pk = torch.frombuffer(bytearray(pks), dtype=torch.uint8).cuda()
        npk = 2 * slh.sizes(param)["n"]
        vit = np.zeros(batch + 8, dtype=slh.VERIFY_DTYPE)
        for i in range(batch):
            vit[i] = (param, 0, items[i]["msg_off"], items[i]["msg_len"], items[i]["sig_off"], kidx[i] * npk)
        bad_sigs = d_s_bad = outs["plain"].clone()
        for j in range(8):
            i = sample[j]
            off = int(items[i]["sig_off"]) + (j * 997) % sb
            bad_sigs[off] ^= 1
            vit[batch + j] = vit[i]
        res = torch.zeros(batch + 8, dtype=torch.int32, device="cuda")
        ctx.verify_batch(vit[:batch], d_m, outs["plain"], d_pk, res)
        torch.cuda.synchronize()
        assert int(res[:batch].sum()) == batch
        res2 = torch.zeros(8, dtype=torch.int32, device="cuda")
        ctx.verify_batch(vit[batch:], d_m, d_s_bad, d_pk, res2)
        torch.cuda.synchronize()
        assert int(res2.sum()) == 0


@pytest.mark.parametrize("param,batch,nkeys", [(1, 32768, 1), (3, 8192, 64)])
def test_batch_beyond_config(slh, param, batch, nkeys):
    """Batches past the benchmarked size (8x for 128f, 2x for 256f with 64
    keys) under a 2 GiB working-memory budget, which the context meets by
    signing the batch in several chunks (about 200 KB of kept chain values
    per 128f signature, 580 KB per 256f one); every mode gives the same
    bytes, sampled signatures equal the oracle's and the whole batch verifies
    on the GPU."""
    import torch
    cfg = 40 + param
    seeds = [workloads.key_seed(param, 100 + i) for i in range(nkeys)]
    keys = oracle_keys(param, seeds)
    assert_gpu_keys(slh, param, seeds, keys)
    kidx = workloads.key_assignment(cfg, batch, nkeys) if nkeys > 1 else [0] * batch
    msgs = workloads.messages(cfg, batch, 32)
    with slh.Context(0, hbm_budget=2 << 30) as ctx:
        first = ctx.add_keys(param, [sk for _, sk in keys])
        items, blob, total = slh.pack_batch([param] * batch, [first + k for k in kidx], msgs)
        d_m = torch.frombuffer(bytearray(blob), dtype=torch.uint8).cuda()
        outs = {}
        for mode in ("plain", "fused", "fused-dedup"):
            d_s = torch.zeros(total, dtype=torch.uint8, device="cuda")
            print("batch", batch, slh.NAMES[param], mode, flush=True)
            ctx.profile(mode == "plain")
            ctx.sign_batch(items, d_m, d_s, mode=slh.MODES[mode])
            torch.cuda.synchronize()
            if mode == "plain":
                ctx.profile(False)
                tree_ms, tree_launches, tree_msgs = ctx.phase_times(reset=True)["tree"]
                assert tree_launches >= 2 and tree_msgs == batch, (tree_launches, tree_msgs)
            outs[mode] = d_s
        for mode in ("fused", "fused-dedup"):
            assert torch.equal(outs[mode], outs["plain"]), mode
        host = outs["plain"].cpu().numpy().tobytes()
        sb = slh.sizes(param)["sig_bytes"]
        sample = workloads.sample_indices(cfg, batch, 16)
        want = oracle_sign_many([(param, keys[kidx[i]][1], msgs[i]) for i in sample])
        for i, w in zip(sample, want):
            got = host[int(items[i]["sig_off"]):int(items[i]["sig_off"]) + sb]
            assert got == w, "item %d: %s" % (i, describe_diff(param, got, w))
        pks = b"".join(pk for pk, _ in keys)
        d_pk = torch.frombuffer(bytearray(pks), dtype=torch.uint8).cuda()
        npk = 2 * slh.sizes(param)["n"]
        vit = np.zeros(batch, dtype=slh.VERIFY_DTYPE)
        vit["param"] = param
        vit["msg_off"] = items["msg_off"]
        vit["msg_len"] = items["msg_len"]
        vit["sig_off"] = items["sig_off"]
        vit["pk_off"] = np.asarray(kidx, dtype=np.uint64) * npk
        res = torch.zeros(batch, dtype=torch.int32, device="cuda")
        ctx.verify_batch(vit, d_m, outs["plain"], d_pk, res)
        torch.cuda.synchronize()
        assert int(res.sum()) == batch
