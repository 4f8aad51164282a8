"""GPU parity of the batched execution modes and of every tuning knob: the
fused persistent kernel, the captured hipGraph (replayed several times with
new message contents, eager work in between), mixed parameter sets in one
launch, every compiled FORS group size, the recompute-WOTS variant, every
compiled kernel shape (FORS leaves per lane and workgroup lanes, TREE block
waves), both layer orders and every instruction variant of the TREE, FORS
and verification kernels all give the oracle's signature, byte for byte."""
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


@pytest.mark.parametrize("schedule", ["default", "chunks"])
def test_graph_mixed_batch_replays(slh, keys, schedule):
    """One captured graph with three parameter-set branches, replayed with new
    message bytes of the same layout; every replay matches the oracle.
    `chunks`: each branch runs the chunk-scheduled fused kernel."""
    import torch
    rng = np.random.default_rng([61, 0])
    with slh.Context(0) as ctx:
        slots = {p: ctx.add_keys(p, keys[p][1]) for p in (1, 2, 3)}
        if schedule == "chunks":
            for p in (1, 2, 3):
                ctx.set_tuning(p, split_max_blocks=slh.SPLIT_NEVER, fused_schedule=slh.FUSED_CHUNKS)
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
                    t = ctx.get_tuning(param)
                    assert {k: t[k] for k in ("fors_trees_per_group", "wgs_per_cu", "keep_chains",
                                              "split_max_blocks")} == {
                        "fors_trees_per_group": fg, "wgs_per_cu": wpc, "keep_chains": keep, "split_max_blocks": split}
                    for mode in ("plain", "fused"):
                        print(NAMES[param], fg, keep, wpc, split, mode, flush=True)
                        got = slh.sign_messages(ctx, [param] * 7, [slot] * 7, msgs, slh.MODES[mode])
                        _check(param, got, want, "fg%d keep%d wpc%d split%d %s" % (fg, keep, wpc, split, mode))


def test_tuning_rejects_uncompiled_variants(slh):
    with slh.Context(0) as ctx:
        for args, knobs in (((1, 3, 0, 1), {}), ((3, 16, 0, 1), {}), ((2, 8, 0, 2), {}),
                            ((1,), {"fors_leaves_per_lane": 8}), ((1,), {"fors_threads": 64}),
                            ((1,), {"tree_waves": 3}), ((1,), {"layer_order": 2}), ((1,), {"variant_tree": 3}),
                            ((1,), {"variant_tree": 1, "tree_waves": 8}),
                            ((2,), {"variant_fors": 2, "fors_leaves_per_lane": 4}),
                            ((3,), {"variant_fors": 1, "fors_threads": 512}),
                            ((7,), {"variant_tree": 1}), ((9,), {"variant_verify": 2}),
                            ((4,), {"tree_waves": 2}), ((5,), {"layer_order": 1}), ((1,), {"fused_wave0_chunks": 1}),
                            ((1,), {"fused_wave0_chunks": 30}), ((3,), {"fused_wave0_chunks": 62}),
                            ((1,), {"fused_waves": 8}), ((4,), {"fused_waves": 2}),
                            ((1,), {"fused_blocks_per_item": 3}), ((5,), {"fused_blocks_per_item": 2}),
                            ((2,), {"fused_blocks_per_item": 2, "fused_wave0_chunks": 97}),
                            ((1,), {"fused_schedule": 3}), ((1,), {"fused_schedule": 2, "fused_waves": 2}),
                            ((2,), {"fused_schedule": 2, "fused_blocks_per_item": 2}),
                            ((3,), {"fused_schedule": 2, "fused_wave0_chunks": 14}), ((4,), {"fused_schedule": 2})):
            with pytest.raises(slh.SlhError) as e:
                ctx.set_tuning(*args, **knobs)
            assert e.value.code == slh.EINVAL, (args, knobs)


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


# every compiled shape of the per-phase kernels and of the fused kernel
SHAPES = [dict(fors_leaves_per_lane=lpl, fors_threads=ft) for lpl in (2, 4) for ft in (128, 256, 512)]


@pytest.mark.parametrize("param", [1, 2, 3, 7])
def test_every_kernel_shape(slh, keys, param):
    """FORS leaves per lane x workgroup lanes for every group size, TREE blocks
    of 2/4/8 waves, in plain and fused mode (the fused kernel takes the leaves
    per lane; its workgroups keep 256 lanes)."""
    sk = keys[param][1] if param in keys else oracle_keys(param, [workloads.key_seed(param, 20)])[0][1]
    msgs = workloads.messages(170 + param, 6, 40)
    want = oracle_sign_many([(param, sk, m) for m in msgs])
    with slh.Context(0) as ctx:
        slot = ctx.add_keys(param, sk)
        for fg in slh.FORS_GROUPS[param]:
            for sh in SHAPES:
                for waves in (2, 4, 8):
                    # the fused kernel takes tree_waves 2/4 as its workgroup size
                    fw = {"fused_waves": waves} if waves != 8 else {}
                    ctx.set_tuning(param, fg, 0, 1, slh.SPLIT_NEVER, tree_waves=waves, **sh, **fw)
                    for mode in ("plain", "fused") if sh["fors_threads"] == 256 and waves != 8 else ("plain",):
                        what = "%s fg%d %s waves%d %s" % (NAMES[param], fg, sh, waves, mode)
                        print(what, flush=True)
                        got = slh.sign_messages(ctx, [param] * 6, [slot] * 6, msgs, slh.MODES[mode])
                        _check(param, got, want, what)


@pytest.mark.parametrize("param", [1, 2, 3, 7])
def test_fused_wave0_share(slh, keys, param):
    """The fused kernel with wave 0 taking fewer or more chains chunks per
    TREE block than the default, across several persistent grids."""
    sk = keys[param][1] if param in keys else oracle_keys(param, [workloads.key_seed(param, 20)])[0][1]
    msgs = workloads.messages(200 + param, 40, 32)
    want = oracle_sign_many([(param, sk, m) for m in msgs])
    L = slh.sizes(param)["len"]
    with slh.Context(0) as ctx:
        slot = ctx.add_keys(param, sk)
        for waves in (4, 2):
            for bpi in (1, 2):
                for w0 in (0, 2, 5, 8, 13, L // 2, L - 6, L + 3, 2 * L - 6):
                    if w0 > bpi * L - 6:
                        continue
                    for wpc in (0, 1):
                        ctx.set_tuning(param, 0, wpc, 1, slh.SPLIT_NEVER, fused_wave0_chunks=w0, fused_waves=waves,
                                       fused_blocks_per_item=bpi)
                        what = "%s fused waves %d bpi %d w0 %d wpc %d" % (NAMES[param], waves, bpi, w0, wpc)
                        print(what, flush=True)
                        got = slh.sign_messages(ctx, [param] * len(msgs), [slot] * len(msgs), msgs,
                                                slh.MODES["fused"])
                        _check(param, got, want, what)


@pytest.mark.parametrize("param", [1, 2, 3, 7, 9])
def test_fused_chunk_schedule(slh, param):
    """The fused kernel scheduled per chains chunk (workgroups take one TREE
    block at a time, its waves take single chunks, a rotating wave finishes
    each block while the others start the next): several keys and ragged
    messages, batches with fewer TREE blocks than workgroups and with several
    blocks per workgroup, kept and recomputed chains, every FORS shape it is
    compiled for, with and without dedup and graph capture."""
    rng = np.random.default_rng([190, param])
    ks = oracle_keys(param, [workloads.key_seed(param, 40 + i) for i in range(3)])
    big = {1: 300, 2: 160, 3: 100, 7: 160, 9: 60}[param]
    with slh.Context(0) as ctx:
        first = ctx.add_keys(param, [sk for _, sk in ks])
        for count in (9, big):
            kidx = [int(rng.integers(0, 3)) for _ in range(count)]
            msgs = [rng.bytes(int(rng.integers(0, 300))) for _ in range(count)]
            want = oracle_sign_many([(param, ks[k][1], m) for k, m in zip(kidx, msgs)])
            for fg in slh.FORS_GROUPS[param]:
                for lpl in (2, 4):
                    for keep in (1, 0):
                        for wpc in (0, 1):
                            if (fg != slh.FORS_GROUPS[param][-1] or lpl != 4) and (keep == 0 or wpc == 1):
                                continue
                            ctx.set_tuning(param, fg, wpc, keep, slh.SPLIT_NEVER, fors_leaves_per_lane=lpl,
                                           fused_schedule=slh.FUSED_CHUNKS)
                            modes = ("fused", "graph", "fused-dedup", "graph-dedup") if keep and not wpc else ("fused",)
                            for mode in modes:
                                what = "%s chunks n%d fg%d lpl%d keep%d wpc%d %s" % (NAMES[param], count, fg, lpl,
                                                                                     keep, wpc, mode)
                                print(what, flush=True)
                                got = slh.sign_messages(ctx, [param] * count, [first + k for k in kidx], msgs,
                                                        slh.MODES[mode])
                                _check(param, got, want, what)


@pytest.mark.parametrize("param", [1, 2, 3, 7, 9])
def test_layers_in_order(slh, keys, param):
    """Layers signed in order (one TREE launch per layer, the WOTS+ signature
    captured as the chains pass the digits) in every mode and block size,
    with kept or recomputed chains requested (in-order keeps nothing), with
    several keys and ragged messages, and a batch larger than one block per
    layer; the dedup modes keep the parallel order."""
    rng = np.random.default_rng([180, param])
    ks = oracle_keys(param, [workloads.key_seed(param, 30 + i) for i in range(3)])
    with slh.Context(0) as ctx:
        first = ctx.add_keys(param, [sk for _, sk in ks])
        for count in (5, 70):
            kidx = [int(rng.integers(0, 3)) for _ in range(count)]
            msgs = [rng.bytes(int(rng.integers(0, 200))) for _ in range(count)]
            want = oracle_sign_many([(param, ks[k][1], m) for k, m in zip(kidx, msgs)])
            for waves in (2, 4, 8):
                for keep in (1, 0):
                    ctx.set_tuning(param, 0, 0, keep, 0, tree_waves=waves, layer_order=slh.LAYERS_IN_ORDER)
                    for mode in ("plain", "fused", "graph", "dedup", "fused-dedup"):
                        if (waves != 4 or keep == 0) and mode not in ("plain", "fused"):
                            continue
                        what = "%s in-order n%d waves%d keep%d %s" % (NAMES[param], count, waves, keep, mode)
                        print(what, flush=True)
                        got = slh.sign_messages(ctx, [param] * count, [first + k for k in kidx], msgs,
                                                slh.MODES[mode])
                        _check(param, got, want, what)


@pytest.mark.parametrize("param", [1, 2, 3])
def test_every_instruction_variant(slh, keys, param):
    """The TREE and FORS kernels in each instruction variant (alone and
    together, plain and in-order, recomputed WOTS), then GPU verification in
    each variant accepting the oracle's signatures and rejecting a corrupted
    one."""
    import torch
    pk, sk = keys[param]
    msgs = workloads.messages(190 + param, 6, 48)
    want = oracle_sign_many([(param, sk, m) for m in msgs])
    with slh.Context(0) as ctx:
        slot = ctx.add_keys(param, sk)
        for vt in (0, 1, 2):
            for vf in (0, 1, 2):
                for order in (slh.LAYERS_PARALLEL, slh.LAYERS_IN_ORDER):
                    for keep in (1, 0):
                        if order == slh.LAYERS_IN_ORDER and keep == 0:
                            continue
                        ctx.set_tuning(param, 0, 0, keep, slh.SPLIT_NEVER, variant_tree=vt, variant_fors=vf,
                                       layer_order=order)
                        what = "%s tree %s fors %s order %d keep %d" % (
                            NAMES[param], slh.VARIANTS[vt], slh.VARIANTS[vf], order, keep)
                        print(what, flush=True)
                        got = slh.sign_messages(ctx, [param] * 6, [slot] * 6, msgs)
                        _check(param, got, want, what)
        sigs = list(want)
        bad = bytearray(sigs[2])
        bad[len(bad) // 2] ^= 0x10
        sigs[2] = bytes(bad)
        sb = slh.sizes(param)["sig_bytes"]
        items = np.zeros(6, dtype=slh.VERIFY_DTYPE)
        mblob = b"".join(msgs)
        off = 0
        for i, m in enumerate(msgs):
            items[i] = (param, 0, off, len(m), i * sb, 0)
            off += len(m)
        d_m = torch.frombuffer(bytearray(mblob), dtype=torch.uint8).cuda()
        d_s = torch.frombuffer(bytearray(b"".join(sigs)), dtype=torch.uint8).cuda()
        d_pk = torch.frombuffer(bytearray(pk), dtype=torch.uint8).cuda()
        for vv in (0, 1, 2):
            ctx.set_tuning(param, variant_verify=vv)
            res = torch.full((6,), -7, dtype=torch.int32, device="cuda")
            print("%s verify %s" % (NAMES[param], slh.VARIANTS[vv]), flush=True)
            ctx.verify_batch(items, d_m, d_s, d_pk, res)
            torch.cuda.synchronize()
            assert res.cpu().tolist() == [1, 1, 0, 1, 1, 1], "verify variant %d" % vv
