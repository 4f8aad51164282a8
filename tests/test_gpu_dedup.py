"""GPU parity of within-batch tree dedup (SLH_MODE_DEDUP).

Messages of one key share the upper hypertree layers (FIPS 205 Algorithm 12:
the layer-j tree is idx_tree >> (j h'), so with h - h' = 63 or 64 bits of
tree address the top layer is one tree and the next ones have 8, 64, ...
trees), and identical messages share every layer.  Each batch here mixes
such repeats with several keys, ragged message lengths and duplicates, and
every dedup mode must give the oracle's signatures byte for byte.  The
number of distinct trees the batch needs is cross-checked from the digests
the oracle computes."""
import numpy as np
import pytest

import oracle
from helpers import NAMES, describe_diff, oracle_keys, oracle_sign_many
from paper_2512_23969_amd import workloads

pytestmark = pytest.mark.gpu

DEDUP_MODES = ("dedup", "fused-dedup", "graph-dedup")


@pytest.fixture(scope="module")
def slh():
    import torch
    assert torch.cuda.is_available()
    from paper_2512_23969_amd import slh as m
    return m


def _batch(param, nkeys, count, seed):
    rng = np.random.default_rng([seed, param])
    keys = oracle_keys(param, [workloads.key_seed(param, 100 + i) for i in range(nkeys)])
    msgs, kidx = [], []
    for i in range(count):
        if i >= 4 and rng.random() < 0.15:  # exact repeat of an earlier (key, message)
            j = int(rng.integers(0, i))
            msgs.append(msgs[j])
            kidx.append(kidx[j])
        else:
            msgs.append(rng.bytes(int(rng.integers(0, 80))))
            kidx.append(int(rng.integers(0, nkeys)))
    return keys, msgs, kidx


def _shared_trees(param, keys, msgs, kidx):
    """(pairs, distinct) of (key, layer, tree) over the batch, from the
    oracle's digest split, for the layers whose tree address has at most 35
    bits (the ones the dedup matches)."""
    p = oracle.params(NAMES[param])
    hp, n = p.hp, p.n
    seen = set()
    pairs = 0
    for m, k in zip(msgs, kidx):
        pk, sk = keys[k]
        r = oracle.prf_msg(p, sk[n:2 * n], pk[:n], m)  # deterministic: opt_rand = PK.seed
        digest = oracle.h_msg(p, r, pk[:n], pk[n:], m)
        _, idx_tree, _ = oracle.split_digest(p, digest)
        for j in range(p.d):
            if p.h - hp - hp * j <= 35:
                pairs += 1
                seen.add((k, j, idx_tree >> (hp * j) if hp * j < 64 else 0))
    return pairs, len(seen)


@pytest.mark.parametrize("param", [1, 2, 3])
def test_dedup_matches_oracle(slh, param):
    keys, msgs, kidx = _batch(param, 3, 48, 7)
    want = oracle_sign_many([(param, keys[k][1], m) for m, k in zip(msgs, kidx)])
    pairs, n_distinct = _shared_trees(param, keys, msgs, kidx)
    assert n_distinct < pairs  # the batch really exercises the sharing
    with slh.Context(0) as ctx:
        first = ctx.add_keys(param, [sk for _, sk in keys])
        d = oracle.params(NAMES[param]).d
        # split 0: this small batch takes the split per-phase path; never:
        # the requested kernels (the fused one in the fused modes)
        for keep, split in ((1, 0), (1, slh.SPLIT_NEVER), (0, slh.SPLIT_NEVER)):
            ctx.set_tuning(param, slh.FORS_GROUPS[param][1], 0, keep, split)
            for mode in DEDUP_MODES:
                print(NAMES[param], mode, "keep", keep, "split", split, flush=True)
                ctx.dedup_stats(reset=True)
                got = slh.sign_messages(ctx, [param] * len(msgs), [first + k for k in kidx], msgs,
                                        slh.MODES[mode])
                for i, (g, w) in enumerate(zip(got, want)):
                    assert g == w, "%s keep%d item %d: %s" % (mode, keep, i, describe_diff(param, g, w))
                # distinct trees computed = ineligible pairs + distinct eligible trees
                trees, distinct = ctx.dedup_stats(reset=True)
                assert trees == len(msgs) * d
                assert distinct == len(msgs) * d - pairs + n_distinct, (trees, distinct, pairs, n_distinct)


def test_dedup_mixed_sets_and_edges(slh):
    """One batch of all three sets; then a one-message batch and a batch of
    the same message repeated (every eligible layer collapses to one tree)."""
    jobs = []
    with slh.Context(0) as ctx:
        slots = {}
        keysets = {}
        for p in (1, 2, 3):
            keysets[p] = oracle_keys(p, [workloads.key_seed(p, 200), workloads.key_seed(p, 201)])
            slots[p] = ctx.add_keys(p, [sk for _, sk in keysets[p]])
        rng = np.random.default_rng(99)
        params, sl, msgs = [], [], []
        for i in range(30):
            p = (1, 2, 3)[i % 3]
            k = int(rng.integers(0, 2))
            params.append(p)
            sl.append(slots[p] + k)
            msgs.append(rng.bytes(int(rng.integers(0, 40))))
            jobs.append((p, keysets[p][k][1], msgs[-1]))
        want = oracle_sign_many(jobs)
        for mode in DEDUP_MODES:
            print("mixed", mode, flush=True)
            got = slh.sign_messages(ctx, params, sl, msgs, slh.MODES[mode])
            for i, (g, w) in enumerate(zip(got, want)):
                assert g == w, "%s item %d: %s" % (mode, i, describe_diff(params[i], g, w))
        for p in (1, 2, 3):
            sk = keysets[p][0][1]
            one = oracle_sign_many([(p, sk, b"single")])[0]
            for mode in DEDUP_MODES:
                print("edge", NAMES[p], mode, flush=True)
                assert slh.sign_messages(ctx, [p], [slots[p]], [b"single"], slh.MODES[mode])[0] == one
                got = slh.sign_messages(ctx, [p] * 9, [slots[p]] * 9, [b"same"] * 9, slh.MODES[mode])
                w = oracle_sign_many([(p, sk, b"same")])[0]
                assert all(g == w for g in got), mode


def test_dedup_rejects_unknown_mode_bits(slh):
    with slh.Context(0) as ctx:
        p = 1
        pk, sk = oracle_keys(p, [workloads.key_seed(p, 300)])[0]
        slot = ctx.add_keys(p, sk)
        with pytest.raises(slh.SlhError):
            slh.sign_messages(ctx, [p], [slot], [b"x"], 8)


def test_graph_dedup_replays(slh):
    """A captured dedup pipeline replayed with new message bytes: the hash
    table, representative list and leaf owners are rebuilt inside the graph
    on every replay, so every replay matches the oracle."""
    import torch
    p = 1
    keys = oracle_keys(p, [workloads.key_seed(p, 150), workloads.key_seed(p, 151)])
    rng = np.random.default_rng(41)
    kidx = [int(rng.integers(0, 2)) for _ in range(40)]
    lens = [int(rng.integers(0, 100)) for _ in range(40)]
    lens[5], kidx[5] = lens[3], kidx[3]  # room for an exact repeat
    with slh.Context(0) as ctx:
        first = ctx.add_keys(p, [sk for _, sk in keys])
        msgs = [rng.bytes(L) for L in lens]
        items, blob, total = slh.pack_batch([p] * 40, [first + k for k in kidx], msgs)
        d_m = torch.zeros(max(1, len(blob)), dtype=torch.uint8, device="cuda")
        d_s = torch.zeros(total, dtype=torch.uint8, device="cuda")
        for rep in range(3):
            msgs = [rng.bytes(L) for L in lens]
            if rep == 2:  # an exact repeat of (key, message) inside the batch
                msgs[5] = msgs[3]
            _, blob2, _ = slh.pack_batch([p] * 40, [first + k for k in kidx], msgs)
            d_m.copy_(torch.frombuffer(bytearray(blob2 or b"\0"), dtype=torch.uint8))
            print("graph-dedup replay", rep, flush=True)
            ctx.sign_batch(items, (d_m.data_ptr(), len(blob)), d_s, slh.MODES["graph-dedup"])
            torch.cuda.synchronize()
            host = d_s.cpu().numpy().tobytes()
            sb = slh.sizes(p)["sig_bytes"]
            want = oracle_sign_many([(p, keys[k][1], m) for k, m in zip(kidx, msgs)])
            for i in range(40):
                o = int(items[i]["sig_off"])
                assert host[o:o + sb] == want[i], "replay %d item %d: %s" % (rep, i, describe_diff(p, host[o:o + sb], want[i]))
            d_s.zero_()
            torch.cuda.synchronize()
