"""Serving parity: requests of mixed parameter sets, keys and lengths served
by the continuous-batching scheduler (several batches in flight, arrivals
while the GPU is busy) give exactly the signature that the same request
signed alone gives, and the oracle's."""
import threading

import numpy as np
import pytest

import oracle
from helpers import NAMES, assert_gpu_keys, describe_diff, oracle_keys, oracle_sign_many
from paper_2512_23969_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slh():
    import torch
    assert torch.cuda.is_available()
    from paper_2512_23969_amd import slh as m
    return m


@pytest.fixture(scope="module")
def keyset(slh):
    """Three oracle keys per set; the GPU's key generation must agree."""
    keys = {}
    for p in (1, 2, 3):
        seeds = [workloads.key_seed(p, 40 + i) for i in range(3)]
        keys[p] = oracle_keys(p, seeds)
        assert_gpu_keys(slh, p, seeds, keys[p])
    return keys


def _mix(n, seed=9):
    reqs = workloads.serving_requests(n, seed=seed, keys_per_set=(3, 3, 3))
    return [p for p, _, _ in reqs], [k for _, k, _ in reqs], [m for _, _, m in reqs]


@pytest.mark.parametrize("schedule", ["default", "chunks"])
def test_replay_equals_alone_and_oracle(slh, keyset, schedule):
    """`chunks`: the server's fused batches run the chunk-scheduled kernel
    (never the split small-batch path), with several lanes in flight."""
    n = 600
    params, kidx, msgs = _mix(n)
    with slh.Server(0, lanes=3, max_batch=128, max_wait_us=500) as srv, slh.Context(0) as ctx:
        slots = {}
        for p in (1, 2, 3):
            slots[p] = srv.add_keys(p, [sk for _, sk in keyset[p]])
            assert ctx.add_keys(p, [sk for _, sk in keyset[p]]) == slots[p]
            if schedule == "chunks":
                srv.set_tuning(p, split_max_blocks=slh.SPLIT_NEVER, fused_schedule=slh.FUSED_CHUNKS)
        ks = [slots[p] + k for p, k in zip(params, kidx)]
        # arrivals at ~ 4x a 128-batch every few ms: batches overlap
        arr = np.cumsum(np.random.default_rng(3).exponential(2e-5, size=n))
        reqs, blob = slh.trace(params, ks, msgs, arr)
        sigs, lat, st = srv.replay(reqs, blob)
        print("serve stats", st, flush=True)
        assert st["completed"] == n and st["launches"] >= 5 and (lat > 0).all()
        served = [sigs[int(r["sig_off"]):int(r["sig_off"]) + slh.sizes(int(r["param"]))["sig_bytes"]].tobytes()
                  for r in reqs]
        # the same requests in one plain batch, and a few truly alone
        batch = slh.sign_messages(ctx, params, ks, msgs)
        for i in range(n):
            assert served[i] == batch[i], "req %d (%s, %d B): %s" % (
                i, NAMES[params[i]], len(msgs[i]), describe_diff(params[i], served[i], batch[i]))
        for i in (0, 1, 2, n // 2, n - 1):
            alone = slh.sign_messages(ctx, [params[i]], [ks[i]], [msgs[i]])[0]
            assert alone == served[i]
    # the oracle on a sample
    sample = list(range(0, n, 50))
    want = oracle_sign_many([(params[i], keyset[params[i]][kidx[i]][1], msgs[i]) for i in sample])
    for i, w in zip(sample, want):
        assert served[i] == w, "req %d: %s" % (i, describe_diff(params[i], served[i], w))


def test_online_submit_poll_two_threads(slh, keyset):
    n = 300
    params, kidx, msgs = _mix(n, seed=13)
    with slh.Server(0, lanes=2, max_batch=64, max_wait_us=300, queue_limit=100000) as srv, \
            slh.Context(0) as ctx:
        slots = {p: srv.add_keys(p, [sk for _, sk in keyset[p]]) for p in (1, 2, 3)}
        for p in (1, 2, 3):
            ctx.add_keys(p, [sk for _, sk in keyset[p]])
        ks = [slots[p] + k for p, k in zip(params, kidx)]
        srv.start()
        results = {}

        def producer(lo, hi):
            for i in range(lo, hi):
                while srv.submit(params[i], ks[i], msgs[i], i) == slh.EBUSY:
                    pass
        th = [threading.Thread(target=producer, args=(0, n // 2)),
              threading.Thread(target=producer, args=(n // 2, n))]
        for t in th:
            t.start()
        import time
        t0 = time.time()
        while len(results) < n and time.time() - t0 < 60:
            for tag, sig, lat in srv.poll(128):
                results[tag] = sig[:slh.sizes(params[tag])["sig_bytes"]]
            time.sleep(0.001)
        for t in th:
            t.join()
        srv.stop()
        for tag, sig, lat in srv.poll(1024):
            results[tag] = sig[:slh.sizes(params[tag])["sig_bytes"]]
        assert len(results) == n
        batch = slh.sign_messages(ctx, params, ks, msgs)
        for i in range(n):
            assert results[i] == batch[i], "req %d" % i


def test_replay_rejects_bad_requests(slh, keyset):
    with slh.Server(0, lanes=1, max_batch=8) as srv:
        slot = srv.add_keys(1, keyset[1][0][1])
        # a SHAKE-128f key: same sizes as SHA2-128f, another set
        other = srv.add_keys(7, oracle_keys(7, [workloads.key_seed(7, 41)])[0][1])
        reqs, blob = slh.trace([1, 1], [slot, slot], [b"a", b"b"], [0.0, 0.0])
        for field, value in (("msg_off", 10 ** 9), ("param", 13), ("key_slot", other + 1),
                             ("key_slot", other), ("arrival_s", -1.0)):
            bad = reqs.copy()
            bad[1][field] = value
            print("bad request", field, value, flush=True)
            with pytest.raises(slh.SlhError):
                srv.replay(bad, blob)
        sigs, lat, st = srv.replay(reqs, blob)  # still serves afterwards
        assert st["completed"] == 2


def test_online_submit_rejects_bad_key_slots(slh, keyset):
    """A request naming a missing key slot, or a slot holding another set's
    key, is refused at submission; the server keeps serving the others."""
    import time
    sk = keyset[1][0][1]
    msgs = [b"x" * 10, b"y" * 20]
    with slh.Server(0, lanes=1, max_batch=8) as srv:
        slot = srv.add_keys(1, sk)
        other = srv.add_keys(7, oracle_keys(7, [workloads.key_seed(7, 41)])[0][1])
        srv.start()
        try:
            for s_bad in (other + 1, other):
                with pytest.raises(slh.SlhError):
                    srv.submit(1, s_bad, b"z", 99)
            for i, m in enumerate(msgs):
                srv.submit(1, slot, m, i)
            got = {}
            t_end = time.time() + 60
            while len(got) < len(msgs) and time.time() < t_end:
                for tag, sig, _ in srv.poll():
                    got[tag] = sig[:slh.sizes(1)["sig_bytes"]]
                time.sleep(0.001)
        finally:
            srv.stop()
        for tag, sig, _ in srv.poll():
            got[tag] = sig[:slh.sizes(1)["sig_bytes"]]
    want = oracle_sign_many([(1, sk, m) for m in msgs])
    assert [got.get(i) for i in range(len(msgs))] == want


def test_serving_mixed_sha2_and_shake(slh):
    """SHA2 and SHAKE keys of the fast and small sets in one served trace,
    several batches in flight: every signature equals the oracle's."""
    params = [1, 7, 2, 8, 9, 3, 10, 4, 7, 1] * 4
    keys = {}
    for p in sorted(set(params)):
        seed = workloads.key_seed(p, 60)
        keys[p] = oracle_keys(p, [seed])[0]
        assert_gpu_keys(slh, p, [seed], [keys[p]])
    rng = np.random.default_rng(61)
    msgs = [rng.bytes(int(rng.integers(0, 400))) for _ in params]
    with slh.Server(0, lanes=3, max_batch=8, max_wait_us=200) as srv:
        slots = {p: srv.add_keys(p, [keys[p][1]]) for p in keys}
        ks = [slots[p] for p in params]
        arr = np.cumsum(np.random.default_rng(62).exponential(1e-4, size=len(params)))
        reqs, blob = slh.trace(params, ks, msgs, arr)
        sigs, lat, st = srv.replay(reqs, blob)
        print("serve stats", st, flush=True)
        assert st["completed"] == len(params) and st["launches"] >= 2
        served = [sigs[int(r["sig_off"]):int(r["sig_off"]) + slh.sizes(int(r["param"]))["sig_bytes"]].tobytes()
                  for r in reqs]
    want = oracle_sign_many([(p, keys[p][1], m) for p, m in zip(params, msgs)])
    for i, (g, w) in enumerate(zip(served, want)):
        assert g == w, "req %d (%s, %d B): %s" % (i, NAMES[params[i]], len(msgs[i]), describe_diff(params[i], g, w))


def test_message_buffer_not_a_multiple_of_four(slh, keyset):
    """A lane message buffer of 4k + 1 bytes filled to its last byte:
    messages start at 4-byte aligned offsets and the last one ends exactly at
    the buffer's end, so the upload must stop there (not at the next
    multiple of four).  Every signature equals the oracle's."""
    sk = keyset[1][0][1]
    rng = np.random.default_rng(77)
    lens = [1001, 1003, 1005, 1081, 7, 4097, 0, 2]
    msgs = [rng.bytes(n) for n in lens]
    with slh.Server(0, lanes=1, max_batch=8, msg_bytes=4097) as srv:
        slot = srv.add_keys(1, sk)
        reqs, blob = slh.trace([1] * len(msgs), [slot] * len(msgs), msgs, [0.0] * len(msgs))
        sigs, lat, st = srv.replay(reqs, blob)
        assert st["completed"] == len(msgs) and st["launches"] >= 2
        served = [sigs[int(r["sig_off"]):int(r["sig_off"]) + slh.sizes(1)["sig_bytes"]].tobytes() for r in reqs]
    want = oracle_sign_many([(1, sk, m) for m in msgs])
    for i, (g, w) in enumerate(zip(served, want)):
        assert g == w, "req %d (%d B): %s" % (i, lens[i], describe_diff(1, g, w))
