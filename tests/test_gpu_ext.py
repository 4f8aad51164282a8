"""GPU parity of the external interface (FIPS 205 Section 10): pure SLH-DSA
with context strings (Algorithm 22), HashSLH-DSA with SHA-256 and SHA-512
(Algorithm 23) and hedged signing (caller-supplied opt_rand), against the
oracle's sign_ext, in the plain, fused and graph-dedup modes."""
import numpy as np
import pytest

import oracle
from helpers import NAMES, describe_diff, oracle_keys
from paper_2512_23969_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slh():
    import torch
    assert torch.cuda.is_available()
    from paper_2512_23969_amd import slh as m
    return m


def _cases(param, rng):
    n = {1: 16, 2: 24, 3: 32}[param]
    mlens = [0, 1, 55, 56, 64, 111, 128, 1000, 20000]
    ctxs = [b"", b"c", bytes(range(255)), rng.bytes(17)]
    out = []
    for i, ml in enumerate(mlens):
        for ph in (0, 1, 2):
            ctx = ctxs[(i + ph) % len(ctxs)]
            rnd = rng.bytes(n) if (i + ph) % 3 == 1 else None
            out.append((rng.bytes(ml), ctx, ph, rnd))
    return out


@pytest.mark.parametrize("param", [1, 2, 3])
def test_ext_matches_oracle(slh, param):
    rng = np.random.default_rng([31, param])
    pk, sk = oracle_keys(param, [workloads.key_seed(param, 700)])[0]
    cases = _cases(param, rng)
    p = oracle.params(NAMES[param])
    want = [oracle.sign_ext(p, m, sk, ctx, ph, rnd) for m, ctx, ph, rnd in cases]
    with slh.Context(0) as ctx:
        slot = ctx.add_keys(param, sk)
        for mode in ("plain", "fused", "graph-dedup"):
            print(NAMES[param], mode, flush=True)
            got = slh.sign_messages_ext(ctx, [param] * len(cases), [slot] * len(cases),
                                        [c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases],
                                        [c[3] for c in cases], slh.MODES[mode])
            for i, (g, w) in enumerate(zip(got, want)):
                m, c, ph, rnd = cases[i]
                assert g == w, "%s case %d (msg %d B, ctx %d B, ph %d, hedged %s): %s" % (
                    mode, i, len(m), len(c), ph, rnd is not None, describe_diff(param, g, w))
    for g, (m, c, ph, rnd) in zip(got, cases):
        assert oracle.verify_ext(p, m, g, pk, c, ph)


@pytest.mark.parametrize("param", [1, 3])
def test_verify_ext_on_gpu(slh, param):
    """GPU verification through the external interface accepts the oracle's
    signatures for their own (context, encoding) and rejects them for any
    other, and rejects a flipped byte."""
    import torch
    rng = np.random.default_rng([37, param])
    pk, sk = oracle_keys(param, [workloads.key_seed(param, 702)])[0]
    p = oracle.params(NAMES[param])
    sb = slh.sizes(param)["sig_bytes"]
    m = rng.bytes(300)
    combos = [(b"", 0), (b"ctx-A", 0), (b"ctx-A", 1), (b"ctx-B", 2)]
    sigs = [oracle.sign_ext(p, m, sk, c, ph) for c, ph in combos]
    blob = bytearray(m)
    coff = {}
    for c, _ in combos:
        coff[c] = len(blob)
        blob += c
    items, expect = [], []
    for si, (c0, ph0) in enumerate(combos):
        for c, ph in combos:
            items.append((param, ph, 0, len(m), si * sb, 0, coff[c], len(c), 0))
            expect.append(int((c, ph) == (c0, ph0)))
    bad = bytearray(sigs[1])
    bad[sb // 2] ^= 0x40
    all_sigs = b"".join(sigs) + bytes(bad)
    c1 = combos[1]
    items.append((param, c1[1], 0, len(m), len(sigs) * sb, 0, coff[c1[0]], len(c1[0]), 0))
    expect.append(0)
    vit = np.array(items, dtype=slh.VERIFY_EXT_DTYPE)
    d_m = torch.frombuffer(bytearray(blob), dtype=torch.uint8).cuda()
    d_s = torch.frombuffer(bytearray(all_sigs), dtype=torch.uint8).cuda()
    d_pk = torch.frombuffer(bytearray(pk), dtype=torch.uint8).cuda()
    res = torch.full((len(items),), -1, dtype=torch.int32, device="cuda")
    with slh.Context(0) as ctx:
        ctx.verify_batch_ext(vit, d_m, d_s, d_pk, res)
        torch.cuda.synchronize()
    assert res.cpu().tolist() == expect


def test_ext_rejects_bad_requests(slh):
    with slh.Context(0) as ctx:
        pk, sk = oracle_keys(1, [workloads.key_seed(1, 701)])[0]
        slot = ctx.add_keys(1, sk)
        for kw in ({"contexts": [bytes(256)]}, {"prehash": [3]}):
            with pytest.raises(slh.SlhError):
                slh.sign_messages_ext(ctx, [1], [slot], [b"m"], **kw)
        # opt_rand outside the message buffer
        items = np.zeros(1, dtype=slh.ITEM_EXT_DTYPE)
        items[0] = (1, slot, 0, 1, 0, 0, 5, 0, 0)
        import torch
        m = torch.zeros(8, dtype=torch.uint8, device="cuda")
        s = torch.zeros(slh.sizes(1)["sig_bytes"], dtype=torch.uint8, device="cuda")
        with pytest.raises(slh.SlhError):
            ctx.sign_batch_ext(items, m, s)
