"""GPU parity of the per-key tree cache (slh_ctx_cache_keys).

The trees of the top hypertree layers depend only on the key (FIPS 205
Algorithm 12: layer d-1-u has 2^(h' u) trees); once cached, signing in a
dedup mode takes their authentication paths and roots from the cache.  A
batch mixing cached and uncached keys, repeats and ragged lengths must give
the oracle's signatures byte for byte, and the dedup statistics must show the
cached layers as not computed."""
import numpy as np
import pytest

import oracle
from helpers import NAMES, describe_diff, oracle_keys, oracle_sign_many
from paper_2512_23969_amd import workloads

pytestmark = pytest.mark.gpu

LAYERS = {1: 4, 2: 3, 3: 2}


@pytest.fixture(scope="module")
def slh():
    import torch
    assert torch.cuda.is_available()
    from paper_2512_23969_amd import slh as m
    return m


def _expected_distinct(param, keys, msgs, kidx, cached):
    """Trees the batch computes: every (message, layer) pair outside the
    cached layers, with eligible triples (tree address of at most 35 bits)
    counted once."""
    p = oracle.params(NAMES[param])
    hp, n = p.hp, p.n
    seen, alone = set(), 0
    for m, k in zip(msgs, kidx):
        pk, sk = keys[k]
        r = oracle.prf_msg(p, sk[n:2 * n], pk[:n], m)
        _, idx_tree, _ = oracle.split_digest(p, oracle.h_msg(p, r, pk[:n], pk[n:], m))
        for j in range(p.d):
            if j + cached.get(k, 0) >= p.d:
                continue
            if p.h - hp - hp * j <= 35:
                seen.add((k, j, idx_tree >> (hp * j) if hp * j < 64 else 0))
            else:
                alone += 1
    return alone + len(seen)


@pytest.mark.parametrize("param", [1, 2, 3])
def test_cached_keys_match_oracle(slh, param):
    keys = oracle_keys(param, [workloads.key_seed(param, 400 + i) for i in range(3)])
    rng = np.random.default_rng([17, param])
    msgs, kidx = [], []
    for i in range(36):
        if i >= 3 and rng.random() < 0.1:
            j = int(rng.integers(0, i))
            msgs.append(msgs[j])
            kidx.append(kidx[j])
        else:
            msgs.append(rng.bytes(int(rng.integers(0, 70))))
            kidx.append(int(rng.integers(0, 3)))
    want = oracle_sign_many([(param, keys[k][1], m) for m, k in zip(msgs, kidx)])
    d = oracle.params(NAMES[param]).d
    with slh.Context(0) as ctx:
        first = ctx.add_keys(param, [sk for _, sk in keys])
        # key 0: the default depth; key 1: one layer; key 2: not cached
        ctx.cache_keys(first, 1, LAYERS[param])
        ctx.cache_keys(first + 1, 1, 1)
        cached = {0: LAYERS[param], 1: 1}
        expect = _expected_distinct(param, keys, msgs, kidx, cached)
        for mode in ("dedup", "fused-dedup", "graph-dedup"):
            print(NAMES[param], mode, flush=True)
            ctx.dedup_stats(reset=True)
            got = slh.sign_messages(ctx, [param] * len(msgs), [first + k for k in kidx], msgs, slh.MODES[mode])
            for i, (g, w) in enumerate(zip(got, want)):
                assert g == w, "%s item %d (key %d): %s" % (mode, i, kidx[i], describe_diff(param, g, w))
            trees, distinct = ctx.dedup_stats(reset=True)
            assert trees == len(msgs) * d
            assert distinct == expect, (distinct, expect)
        # the cache is ignored outside the dedup modes
        got = slh.sign_messages(ctx, [param] * len(msgs), [first + k for k in kidx], msgs, slh.MODES["plain"])
        assert got == want


def test_cache_arguments(slh):
    with slh.Context(0) as ctx:
        k1 = oracle_keys(1, [workloads.key_seed(1, 500), workloads.key_seed(1, 501)])
        k3 = oracle_keys(3, [workloads.key_seed(3, 500)])
        a = ctx.add_keys(1, [sk for _, sk in k1])
        b = ctx.add_keys(3, [sk for _, sk in k3])
        for first, count, layers in ((a, 1, 0), (a, 1, 7), (b, 1, 5), (a, 3, 2), (b, 2, 1), (a, 0, 1)):
            with pytest.raises(slh.SlhError):
                ctx.cache_keys(first, count, layers)
        ctx.cache_keys(a, 2, 2)
        with pytest.raises(slh.SlhError):
            ctx.cache_keys(a + 1, 1, 2)  # cached already
        ctx.cache_keys(b, 1, 4)


@pytest.mark.parametrize("cache_layers", [3, 5])
def test_server_with_cache(slh, cache_layers):
    """Replay through a server whose lanes cache the keys' upper layers; the
    layer count is clamped to each set's limit (4 for the h' = 4 sets, none
    for the small sets)."""
    import torch  # noqa: F401
    params = [1, 2, 3, 1, 1, 3, 2, 1] + ([9, 4, 9] if cache_layers == 5 else [])
    sets = sorted(set(params))
    keysets = {p: oracle_keys(p, [workloads.key_seed(p, 600)]) for p in sets}
    rng = np.random.default_rng(23)
    msgs = [rng.bytes(int(rng.integers(1, 300))) for _ in params]
    with slh.Server(0, lanes=2, mode=slh.MODES["fused-dedup"], cache_layers=cache_layers) as srv:
        slots = {p: srv.add_keys(p, keysets[p][0][1]) for p in sets}
        reqs, blob = slh.trace(params, [slots[p] for p in params], msgs, [0.0] * len(params))
        sigs, lat, st = srv.replay(reqs, blob)
    want = oracle_sign_many([(p, keysets[p][0][1], m) for p, m in zip(params, msgs)])
    for i, p in enumerate(params):
        o = int(reqs[i]["sig_off"])
        got = sigs[o:o + slh.sizes(p)["sig_bytes"]].tobytes()
        assert got == want[i], "request %d: %s" % (i, describe_diff(p, got, want[i]))
