"""Calls on one context return without waiting for the GPU: two signing calls
in a row are both queued while the first still runs (the host waits only
for the call two before, whose pinned item copy it reuses), on one stream
and on two streams (the second call is then ordered after the first on the
GPU, since they share the context's working memory).  Both batches equal the
oracle's signatures byte for byte."""
import pytest

from helpers import describe_diff, oracle_keys, oracle_sign_many
from paper_2512_23969_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slh():
    import torch
    assert torch.cuda.is_available()
    from paper_2512_23969_amd import slh as m
    return m


@pytest.mark.parametrize("streams", [1, 2])
def test_two_calls_in_flight(slh, streams):
    import time
    import torch
    param, batch = 1, 1024
    pk, sk = oracle_keys(param, [workloads.key_seed(param, 7)])[0]
    msgs = [workloads.messages(60 + j, batch, 32) for j in range(2)]
    with slh.Context(0) as ctx:
        slot = ctx.add_keys(param, sk)
        packed = [slh.pack_batch([param] * batch, [slot] * batch, m) for m in msgs]
        d_m = [torch.frombuffer(bytearray(p[1]), dtype=torch.uint8).cuda() for p in packed]
        d_s = [torch.zeros(p[2], dtype=torch.uint8, device="cuda") for p in packed]
        st = [torch.cuda.Stream() for _ in range(streams)]
        # warm-up: working memory and pinned copies of both call slots exist
        for j in range(2):
            ctx.sign_batch(packed[j][0], d_m[j], d_s[j], stream=st[j % streams])
        torch.cuda.synchronize()
        # one batch's GPU time
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st[0])
        ctx.sign_batch(packed[0][0], d_m[0], d_s[0], stream=st[0])
        e1.record(st[0])
        torch.cuda.synchronize()
        gpu_ms = e0.elapsed_time(e1)
        for t in d_s:
            t.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(2):
            ctx.sign_batch(packed[j][0], d_m[j], d_s[j], stream=st[j % streams])
        host_ms = 1e3 * (time.perf_counter() - t0)
        busy = not all(s.query() for s in st)
        torch.cuda.synchronize()
        print("streams %d: two calls queued in %.3f ms, one batch takes %.3f ms on the GPU, busy after: %s"
              % (streams, host_ms, gpu_ms, busy), flush=True)
        assert host_ms < 0.5 * gpu_ms, "the calls waited for the GPU"
        assert busy, "the GPU had finished before the second call returned"
        out = [t.cpu().numpy().tobytes() for t in d_s]
    sb = slh.sizes(param)["sig_bytes"]
    for j in range(2):
        want = oracle_sign_many([(param, sk, m) for m in msgs[j]])
        items = packed[j][0]
        for i, w in enumerate(want):
            got = out[j][int(items[i]["sig_off"]):int(items[i]["sig_off"]) + sb]
            assert got == w, "batch %d item %d: %s" % (j, i, describe_diff(param, got, w))
