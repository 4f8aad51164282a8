"""The signing entry point that allocates nothing (slh_sign_batch_noalloc).

It is called through the C ABI and compared with slh_sign_batch, the entry
point it is a variant of, byte for byte: two calls in a row, the second with
a smaller batch, in every mode it accepts; a batch larger than one chunk of
the fixed working array (signed in several chunks); a sample of each batch
also equals the oracle's signatures.  Argument errors are refused before
anything is written."""
import numpy as np
import pytest

from helpers import describe_diff, oracle_keys, oracle_sign_many
from paper_2512_23969_amd import workloads

pytestmark = pytest.mark.gpu

SETS = (1, 2, 3)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2512_23969_amd import slh
    keys = {p: oracle_keys(p, [workloads.key_seed(p, 40 + i) for i in range(2)]) for p in SETS}
    ctx = slh.Context(0)
    slots = {p: ctx.add_keys(p, [sk for _, sk in keys[p]]) for p in SETS}
    yield slh, ctx, keys, slots
    ctx.close()


def make_batch(slots, spec, seed):
    """spec: [(param, count)]; keys alternate over two slots; message
    lengths 0..299 bytes."""
    rng = np.random.default_rng([seed, 0x0A11])
    params, ks, kidx, msgs = [], [], [], []
    for p, cnt in spec:
        for _ in range(cnt):
            k = int(rng.integers(0, 2))
            params.append(p)
            ks.append(slots[p] + k)
            kidx.append(k)
            msgs.append(rng.bytes(int(rng.integers(0, 300))))
    return params, ks, kidx, msgs


def sign_both(slh, ctx, params, ks, msgs, mode):
    """(items, bytes from slh_sign_batch_noalloc, bytes from slh_sign_batch)."""
    import torch
    items, blob, total = slh.pack_batch(params, ks, msgs)
    d_m = torch.frombuffer(bytearray(blob or b"\0"), dtype=torch.uint8).cuda()
    got = torch.full((total,), 0xAB, dtype=torch.uint8, device="cuda")
    want = torch.zeros(total, dtype=torch.uint8, device="cuda")
    ctx.sign_batch_noalloc(items, (d_m.data_ptr(), len(blob)), got, mode=mode)
    ctx.sign_batch(items, (d_m.data_ptr(), len(blob)), want, mode=mode)
    torch.cuda.synchronize()
    return items, got.cpu().numpy().tobytes(), want.cpu().numpy().tobytes()


def check(slh, keys, params, kidx, msgs, items, got, want, sample):
    for i, it in enumerate(items):
        p, o = int(it["param"]), int(it["sig_off"])
        sb = slh.sizes(p)["sig_bytes"]
        assert got[o:o + sb] == want[o:o + sb], "request %d (%s): %s" % (
            i, slh.NAMES[p], describe_diff(p, got[o:o + sb], want[o:o + sb]))
    idx = sorted(set(sample))
    ref = oracle_sign_many([(params[i], keys[params[i]][kidx[i]][1], msgs[i]) for i in idx])
    for i, r in zip(idx, ref):
        o = int(items[i]["sig_off"])
        assert got[o:o + len(r)] == r, "request %d differs from the oracle" % i


def first_last(params):
    out = []
    for p in SETS:
        pos = [i for i, q in enumerate(params) if q == p]
        if pos:
            out += [pos[0], pos[-1]]
    return out


@pytest.mark.parametrize("mode", ["plain", "fused", "dedup", "fused-dedup"])
def test_two_calls_equal_sign_batch(env, mode):
    slh, ctx, keys, slots = env
    m = slh.MODES[mode]
    for call, spec in enumerate(([(1, 300), (2, 100), (3, 60)], [(1, 40), (3, 5)])):
        print("no-alloc %s call %d: %s" % (mode, call, spec), flush=True)
        params, ks, kidx, msgs = make_batch(slots, spec, 10 * call + len(mode))
        items, got, want = sign_both(slh, ctx, params, ks, msgs, m)
        check(slh, keys, params, kidx, msgs, items, got, want, first_last(params))


def test_chunk_scheduled_fused(env):
    """The fused kernel scheduled per chains chunk, in both fused modes, on
    two calls in a row."""
    slh, ctx, keys, slots = env
    try:
        for p in SETS:
            ctx.set_tuning(p, fused_schedule=slh.FUSED_CHUNKS)
        for mode in ("fused", "fused-dedup"):
            for call, spec in enumerate(([(1, 300), (2, 100), (3, 60)], [(1, 40), (3, 5)])):
                print("no-alloc chunk-scheduled %s call %d: %s" % (mode, call, spec), flush=True)
                params, ks, kidx, msgs = make_batch(slots, spec, 30 + 10 * call + len(mode))
                items, got, want = sign_both(slh, ctx, params, ks, msgs, slh.MODES[mode])
                check(slh, keys, params, kidx, msgs, items, got, want, first_last(params))
    finally:
        for p in SETS:
            ctx.set_tuning(p)


def test_several_chunks(env):
    """400 requests of 256f need about 470 MB of working memory in plain mode
    with kept chains: more than the array holds, so they run in chunks."""
    slh, ctx, keys, slots = env
    for call, cnt in enumerate((400, 100)):
        print("no-alloc chunked call %d: %d x 256f" % (call, cnt), flush=True)
        params, ks, kidx, msgs = make_batch(slots, [(3, cnt)], 77 + call)
        items, got, want = sign_both(slh, ctx, params, ks, msgs, slh.MODE_PLAIN)
        # first and last request, and the two around the first chunk boundary
        check(slh, keys, params, kidx, msgs, items, got, want, [0, min(228, cnt - 1), min(229, cnt - 1), cnt - 1])


def test_refused_before_anything_runs(env):
    import torch
    slh, ctx, keys, slots = env
    params, ks, kidx, msgs = make_batch(slots, [(1, 3)], 5)
    items, blob, total = slh.pack_batch(params, ks, msgs)
    d_m = torch.frombuffer(bytearray(blob), dtype=torch.uint8).cuda()
    out = torch.full((total,), 0xAB, dtype=torch.uint8, device="cuda")
    with pytest.raises(slh.SlhError) as e:
        ctx.sign_batch_noalloc(items, (d_m.data_ptr(), len(blob)), out, mode=slh.MODES["graph"])
    assert e.value.code == slh.EINVAL
    big = np.resize(items, slh.NOALLOC_MAX_ITEMS + 1)
    with pytest.raises(slh.SlhError) as e:
        ctx.sign_batch_noalloc(big, (d_m.data_ptr(), len(blob)), out)
    assert e.value.code == slh.EINVAL
    bad = items.copy()
    bad["key_slot"][1] = 10_000
    with pytest.raises(slh.SlhError) as e:
        ctx.sign_batch_noalloc(bad, (d_m.data_ptr(), len(blob)), out)
    assert e.value.code == slh.EINVAL
    torch.cuda.synchronize()
    assert bool((out == 0xAB).all()), "a refused call wrote signature bytes"
