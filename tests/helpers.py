"""Shared test helpers: oracle fan-out over host threads and signature diffs."""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import oracle

NAMES = {1: "128f", 2: "192f", 3: "256f", 4: "128s", 5: "192s", 6: "256s",
         7: "shake-128f", 8: "shake-192f", 9: "shake-256f", 10: "shake-128s", 11: "shake-192s",
         12: "shake-256s"}


def host_threads() -> int:
    # at most 16 host threads: the share of host cores a one-GPU machine gives one process
    return max(1, min(16, os.cpu_count() or 1))


def oracle_keys(param: int, seeds):
    """(pk, sk) of each seed from the oracle's key generation, in parallel."""
    p = oracle.params(NAMES[param])
    with ThreadPoolExecutor(host_threads()) as ex:
        return list(ex.map(lambda s: oracle.keygen(p, s), seeds))


def assert_gpu_keys(slh, param: int, seeds, keys):
    """slh.keygen (the HIP path) gives the oracle's (pk, sk) for every seed."""
    for i, (seed, want) in enumerate(zip(seeds, keys)):
        assert slh.keygen(param, seed) == want, "%s key %d: GPU keygen differs from the oracle" % (
            NAMES[param], i)


def oracle_sign_many(jobs):
    """jobs: list of (param, sk, msg) -> list of signatures, in parallel
    (the ctypes call releases the GIL)."""
    def one(job):
        param, sk, msg = job
        return oracle.sign(oracle.params(NAMES[param]), msg, sk)
    with ThreadPoolExecutor(host_threads()) as ex:
        return list(ex.map(one, jobs))


def segments(param: int):
    """Named byte ranges of a signature: R, FORS tree t, layer j WOTS / auth."""
    p = oracle.params(NAMES[param])
    n = p.n
    out = [("R", 0, n)]
    off = n
    for t in range(p.k):
        out.append(("fors_sk[%d]" % t, off, off + n))
        out.append(("fors_auth[%d]" % t, off + n, off + (p.a + 1) * n))
        off += (p.a + 1) * n
    for j in range(p.d):
        out.append(("wots[%d]" % j, off, off + p.len * n))
        out.append(("xmss_auth[%d]" % j, off + p.len * n, off + (p.len + p.hp) * n))
        off += (p.len + p.hp) * n
    assert off == oracle.sig_bytes(p)
    return out


def describe_diff(param: int, got: bytes, want: bytes, limit: int = 12) -> str:
    if len(got) != len(want):
        return "length %d != %d" % (len(got), len(want))
    bad = [name for name, a, b in segments(param) if got[a:b] != want[a:b]]
    if not bad:
        return "identical"
    return "%d segments differ: %s%s" % (len(bad), ", ".join(bad[:limit]), " ..." if len(bad) > limit else "")
